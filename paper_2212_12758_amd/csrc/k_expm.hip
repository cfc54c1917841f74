// exp(alpha H_hat) e_1 by scaling and squaring with a diagonal Pade
// approximant r_q (Higham, SIAM J. Matrix Anal. Appl. 26 (2005) 1179-1193),
// the matrix exponential the paper applies to the compressed matrix (Section 5
// experiments).  The degree q in {3,5,7,9,13} and the scaling 2^-s follow from
// ||alpha H_hat||_1 and the published theta_q bounds.
//
// The matrix products are spread over many workgroups.  Every degree is
// evaluated through the degree-13 scheme
//     U = A [A6 (c13 A6 + c11 A4 + c9 A2) + c7 A6 + c5 A4 + c3 A2 + c1 I]
//     V =    A6 (c12 A6 + c10 A4 + c8 A2) + c6 A6 + c4 A4 + c2 A2 + c0 I
// with c_j = 0 for j > q, so the launch sequence does not depend on q and can
// be captured once:
//   k_exp_prep        ||alpha H_hat||_1, q, s, coefficients, A = alpha 2^-s H_hat
//   k_exp_gemm<1..5>  A2, A4, A6 (+ the two inner sums), U-inner and V, P and Q
//   k_exp_solve       LU of Q = V - U with partial pivoting, x = Q^{-1} P e_1,
//                     then the squaring phase X^(2^s) e_1 for X = Q^{-1} P.
// Workspace slots (m x m each, column-major, ld = m_used): 0 A, 1 A2, 2 A4,
// 3 A6, 4 T1 -> P, 5 T1' -> Q, 6 T2 -> X, 7 V -> squaring buffer.
#include "fab_dev.h"

namespace fab {

namespace {

constexpr int ET = 16;     // GEMM output tile (ET x ET per workgroup, one output per thread)
constexpr int EK = 64;     // k-chunk staged in LDS
constexpr int LDSM = 112;  // LU factors kept in LDS up to this order
constexpr int EMAXM = 512;
constexpr int VEC_SQ = 5;  // squarings up to this count are applied to the vector

__device__ inline int exp_mused(const SolveDev& d, int q) { return d.status[4 + 2 * q]; }

// parameter block behind the vectors: [0] q, [1] s, [2] scale, [3] ||alpha H||_1, [4..17] c_j
__device__ inline double* exp_params(const DenseDev& g, double* ws) { return ws + g.oVec + 4 * (long long)(g.m + 1); }

__device__ inline double pade_c(int q, int j) {
  // c_j = (2q-j)! q! / ((2q)! j! (q-j)!), built as a running product
  double c = 1.0;
  for (int i = 0; i < j; ++i) c *= (double)(q - i) / (double)((2 * q - i) * (i + 1));
  return c;
}

__device__ inline double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

}  // namespace

// one workgroup per right-hand side
__global__ void __launch_bounds__(256) k_exp_prep(SolveDev d, DenseDev g) {
  const int q = blockIdx.x, tid = threadIdx.x;
  double* ws = g.base + (long long)q * g.stride;
  const int m = exp_mused(d, q);
  __shared__ double sh[4];
  if (m == 0) return;
  const double* Hh = ws + g.oH;
  double cmax = 0.0;
  for (int c = tid; c < m; c += 256) {
    double sacc = 0.0;
    for (int r = 0; r < m; ++r) sacc += fabs(Hh[r + (long long)c * m]);
    cmax = fmax(cmax, sacc);
  }
  for (int off = 32; off >= 1; off >>= 1) cmax = fmax(cmax, __shfl_xor(cmax, off, 64));
  if ((tid & 63) == 0) sh[tid >> 6] = cmax;
  __syncthreads();
  const double nrm = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3])) * fabs(g.alpha);
  const double theta[5] = {1.495585217958292e-2, 2.539398330063230e-1, 9.504178996162932e-1,
                           2.097847961257068e0, 5.371920351148152e0};
  const int degs[5] = {3, 5, 7, 9, 13};
  int qd = 13, ssq = 0;
  for (int t = 0; t < 4; ++t)
    if (nrm <= theta[t]) { qd = degs[t]; break; }
  if (qd == 13 && nrm > theta[4]) ssq = (int)ceil(log2(nrm / theta[4]));
  if (ssq < 0) ssq = 0;
  const double scale = g.alpha * ldexp(1.0, -ssq);
  double* P = exp_params(g, ws);
  if (tid < 14) P[4 + tid] = tid <= qd ? pade_c(qd, tid) : 0.0;
  if (tid == 0) {
    P[0] = qd;
    P[1] = ssq;
    P[2] = scale;
    P[3] = nrm;
  }
  double* A = ws + g.oM;
  const long long mm = (long long)m * m;
  for (long long x = tid; x < mm; x += 256) A[x] = scale * Hh[x];
}

// One ET x ET output tile per workgroup: C = X Y (and C2 = X Y2 in pass 4),
// k staged through LDS in chunks of EK; the elementwise sums of the scheme are
// fused into the store.
template <int MODE>
__global__ void __launch_bounds__(256) k_exp_gemm(SolveDev d, DenseDev g) {
  const int q = blockIdx.z;
  double* ws = g.base + (long long)q * g.stride;
  const int m = exp_mused(d, q);
  const int i0 = blockIdx.x * ET, j0 = blockIdx.y * ET;
  if (m == 0 || i0 >= m || j0 >= m) return;
  const long long mm = (long long)m * m;
  double* S0 = ws + g.oM;
  const double* X;
  const double* Y;
  const double* Y2 = nullptr;
  if (MODE == 1) { X = S0; Y = S0; }
  else if (MODE == 2) { X = S0 + mm; Y = S0 + mm; }
  else if (MODE == 3) { X = S0 + 2 * mm; Y = S0 + mm; }
  else if (MODE == 4) { X = S0 + 3 * mm; Y = S0 + 4 * mm; Y2 = S0 + 5 * mm; }
  else { X = S0; Y = S0 + 6 * mm; }
  __shared__ double Xs[EK][ET];
  __shared__ double Ys[ET][EK + 1];
  __shared__ double Y2s[MODE == 4 ? ET : 1][EK + 1];
  const int tid = threadIdx.x;
  const int ii = tid & (ET - 1), jj = tid >> 4;
  double a1 = 0.0, a2 = 0.0;
  for (int k0 = 0; k0 < m; k0 += EK) {
    // X chunk: rows i0..i0+15, columns k0..k0+63 -> Xs[k][i]
#pragma unroll
    for (int t = 0; t < EK * ET / 256; ++t) {
      const int kk = jj + 16 * t;
      const int r = i0 + ii, k = k0 + kk;
      Xs[kk][ii] = (r < m && k < m) ? X[r + (long long)k * m] : 0.0;
    }
    // Y chunk: rows k0..k0+63, columns j0..j0+15 -> Ys[j][k]
#pragma unroll
    for (int t = 0; t < EK * ET / 256; ++t) {
      const int e = tid + 256 * t;
      const int kk = e & (EK - 1), jc = e >> 6;
      const int k = k0 + kk, c = j0 + jc;
      const bool ok = k < m && c < m;
      Ys[jc][kk] = ok ? Y[k + (long long)c * m] : 0.0;
      if (MODE == 4) Y2s[jc][kk] = ok ? Y2[k + (long long)c * m] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < EK; ++kk) {
      const double xv = Xs[kk][ii];
      a1 += xv * Ys[jj][kk];
      if (MODE == 4) a2 += xv * Y2s[jj][kk];
    }
    __syncthreads();
  }
  const int i = i0 + ii, j = j0 + jj;
  if (i >= m || j >= m) return;
  const long long o = i + (long long)j * m;
  const double* c = exp_params(g, ws) + 4;
  const double I = i == j ? 1.0 : 0.0;
  if (MODE == 1) {
    S0[mm + o] = a1;                                   // A2
  } else if (MODE == 2) {
    S0[2 * mm + o] = a1;                               // A4
  } else if (MODE == 3) {
    const double A2 = S0[mm + o], A4 = S0[2 * mm + o];
    S0[3 * mm + o] = a1;                               // A6
    S0[4 * mm + o] = c[13] * a1 + c[11] * A4 + c[9] * A2;
    S0[5 * mm + o] = c[12] * a1 + c[10] * A4 + c[8] * A2;
  } else if (MODE == 4) {
    const double A2 = S0[mm + o], A4 = S0[2 * mm + o], A6 = S0[3 * mm + o];
    S0[6 * mm + o] = a1 + c[7] * A6 + c[5] * A4 + c[3] * A2 + c[1] * I;   // inner factor of U
    S0[7 * mm + o] = a2 + c[6] * A6 + c[4] * A4 + c[2] * A2 + c[0] * I;   // V
  } else {
    const double V = S0[7 * mm + o];
    S0[4 * mm + o] = V + a1;                           // P = V + U
    S0[5 * mm + o] = V - a1;                           // Q = V - U
  }
}

// Solve L U x = b (row permutation perm applied on load) with one wave; rows
// r = lane + 64 u live in registers, the pivot element of each step is read
// from its owner lane with readlane, so the substitutions need no barrier.
template <int R>
__device__ void wave_lu_solve(int m, const double* LU, const int* perm, const double* b, double* out) {
  const int lane = threadIdx.x & 63;
  double x[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int r = lane + 64 * u;
    x[u] = r < m ? b[perm[r]] : 0.0;
  }
  for (int j = 0; j < m; ++j) {
    const int uj = j >> 6;
    double src = x[0];
#pragma unroll
    for (int u = 1; u < R; ++u)
      if (uj == u) src = x[u];
    const double xj = readlane_d(src, j & 63);
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int r = lane + 64 * u;
      if (r > j && r < m) x[u] -= LU[r + (long long)j * m] * xj;
    }
  }
  for (int j = m - 1; j >= 0; --j) {
    const int uj = j >> 6;
    double src = x[0];
#pragma unroll
    for (int u = 1; u < R; ++u)
      if (uj == u) src = x[u];
    const double xj = readlane_d(src, j & 63) / LU[j + (long long)j * m];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int r = lane + 64 * u;
      if (r == j) x[u] = xj;
      else if (r < j) x[u] -= LU[r + (long long)j * m] * xj;
    }
  }
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int r = lane + 64 * u;
    if (r < m) out[r] = x[u];
  }
}

__device__ void lu_solve_any(int m, const double* LU, const int* perm, const double* b, double* out) {
  if (m <= 128) wave_lu_solve<2>(m, LU, perm, b, out);
  else if (m <= 256) wave_lu_solve<4>(m, LU, perm, b, out);
  else wave_lu_solve<8>(m, LU, perm, b, out);
}

// C = X X by one workgroup (squaring phase when s > VEC_SQ); global operands.
__device__ void block_square(int m, const double* X, double* C, double (*Xs)[ET], double (*Ys)[EK + 1]) {
  const int tid = threadIdx.x, ii = tid & (ET - 1), jj = tid >> 4;
  const int nt = (m + ET - 1) / ET;
  for (int ti = 0; ti < nt; ++ti)
    for (int tj = 0; tj < nt; ++tj) {
      const int i0 = ti * ET, j0 = tj * ET;
      double a = 0.0;
      for (int k0 = 0; k0 < m; k0 += EK) {
        for (int u = 0; u < EK * ET / 256; ++u) {
          const int kk = jj + 16 * u, r = i0 + ii, k = k0 + kk;
          Xs[kk][ii] = (r < m && k < m) ? X[r + (long long)k * m] : 0.0;
          const int e = tid + 256 * u, kk2 = e & (EK - 1), jc = e >> 6;
          const int k2 = k0 + kk2, c = j0 + jc;
          Ys[jc][kk2] = (k2 < m && c < m) ? X[k2 + (long long)c * m] : 0.0;
        }
        __syncthreads();
        for (int kk = 0; kk < EK; ++kk) a += Xs[kk][ii] * Ys[jj][kk];
        __syncthreads();
      }
      const int i = i0 + ii, j = j0 + jj;
      if (i < m && j < m) C[i + (long long)j * m] = a;
    }
  __syncthreads();
}

__global__ void __launch_bounds__(256) k_exp_solve(SolveDev d, DenseDev g) {
  const int q = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  double* ws = g.base + (long long)q * g.stride;
  const int m = exp_mused(d, q);
  if (m == 0) return;
  const long long mm = (long long)m * m;
  double* S0 = ws + g.oM;
  const double* Pm = S0 + 4 * mm;
  double* Qg = S0 + 5 * mm;
  double* c = ws + g.oVec;
  double* info = ws + g.oInfo;
  const int ssq = (int)exp_params(g, ws)[1];
  extern __shared__ double lu_lds[];
  __shared__ int perm[EMAXM];
  __shared__ double prow[EMAXM], jrow[EMAXM], lcol[EMAXM], xs[EMAXM], xt[EMAXM];
  __shared__ double Xs[EK][ET];
  __shared__ double Ys[ET][EK + 1];
  __shared__ int sp, sing;
  // the dynamic LDS is sized for the planned order d.m (m_used <= d.m)
  const bool in_lds = d.m <= LDSM;
  double* L = in_lds ? lu_lds : Qg;
  if (in_lds)
    for (long long x = tid; x < mm; x += 256) L[x] = Qg[x];
  for (int r = tid; r < m; r += 256) perm[r] = r;
  if (tid == 0) sing = 0;
  __syncthreads();

  // LU with partial pivoting.  Per column: wave 0 finds the pivot, snapshots
  // the pivot row and row j, forms the multipliers and records the row
  // exchange; then every thread updates the trailing block (the exchange of
  // rows j and p is folded into that update) and swaps the multipliers of
  // rows j and p left of column j.
  for (int j = 0; j < m; ++j) {
    if (wid == 0) {
      double best = -1.0;
      int bi = j;
      for (int r = j + lane; r < m; r += 64) {
        const double v = fabs(L[r + (long long)j * m]);
        if (v > best) { best = v; bi = r; }
      }
      for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      const int p = bi;
      for (int cc = j + lane; cc < m; cc += 64) {
        prow[cc] = L[p + (long long)cc * m];
        jrow[cc] = L[j + (long long)cc * m];
      }
      const double pv = L[p + (long long)j * m];
      const double ajj = L[j + (long long)j * m];
      for (int r = j + 1 + lane; r < m; r += 64) {
        const double ar = (r == p) ? ajj : L[r + (long long)j * m];
        lcol[r] = pv != 0.0 ? ar / pv : 0.0;
      }
      if (lane == 0) {
        sp = p;
        if (p != j) {
          const int t = perm[j];
          perm[j] = perm[p];
          perm[p] = t;
        }
        if (pv == 0.0) sing = 1;
      }
    }
    __syncthreads();
    const int p = sp;
    if (p != j)
      for (int cc = tid; cc < j; cc += 256) {
        const double t = L[j + (long long)cc * m];
        L[j + (long long)cc * m] = L[p + (long long)cc * m];
        L[p + (long long)cc * m] = t;
      }
    for (int cc = j + wid; cc < m; cc += 4) {
      const double pc = prow[cc], jc = jrow[cc];
      for (int r = j + lane; r < m; r += 64) {
        double v;
        if (r == j) v = pc;
        else if (cc == j) v = lcol[r];
        else v = ((r == p) ? jc : L[r + (long long)cc * m]) - lcol[r] * pc;
        L[r + (long long)cc * m] = v;
      }
    }
    __syncthreads();
  }

  if (ssq == 0) {
    // x = Q^{-1} (P e_1)
    if (wid == 0) lu_solve_any(m, L, perm, Pm, c);
  } else {
    // X = Q^{-1} P column by column (one wave per column), into slot 6
    double* X = S0 + 6 * mm;
    for (int cc = wid; cc < m; cc += 4) lu_solve_any(m, L, perm, Pm + (long long)cc * m, X + (long long)cc * m);
    __syncthreads();
    int vec = ssq;
    if (ssq > VEC_SQ) {
      // leading squarings as matrix products, the last VEC_SQ on the vector
      double* Xa = X;
      double* Xb = S0 + 7 * mm;
      for (int t = 0; t < ssq - VEC_SQ; ++t) {
        block_square(m, Xa, Xb, Xs, Ys);
        double* tt = Xa;
        Xa = Xb;
        Xb = tt;
      }
      X = Xa;
      vec = VEC_SQ;
    }
    // x <- X^(2^vec) e_1 by 2^vec products with the vector
    for (int r = tid; r < m; r += 256) xs[r] = X[r];
    __syncthreads();
    const int reps = (1 << vec) - 1;
    for (int t = 0; t < reps; ++t) {
      for (int r = tid; r < m; r += 256) {
        double a = 0.0;
        for (int cc = 0; cc < m; ++cc) a += X[r + (long long)cc * m] * xs[cc];
        xt[r] = a;
      }
      __syncthreads();
      for (int r = tid; r < m; r += 256) xs[r] = xt[r];
      __syncthreads();
    }
    for (int r = tid; r < m; r += 256) c[r] = xs[r];
  }
  if (tid == 0) {
    info[4] = ssq;                   // number of squarings
    info[6] = exp_params(g, ws)[3];  // ||alpha H_hat||_1
    if (sing) info[3] = 1.0;         // singular Pade denominator
  }
}

size_t exp_solve_lds(int m) { return m <= LDSM ? (size_t)m * m * 8 : 0; }

hipError_t exp_launch(const SolveDev& d, const DenseDev& g, hipStream_t st) {
  const int m = d.m;
  const dim3 grid((m + ET - 1) / ET, (m + ET - 1) / ET, d.nrhs);
  hipLaunchKernelGGL(k_exp_prep, dim3(d.nrhs), dim3(256), 0, st, d, g);
  hipLaunchKernelGGL(k_exp_gemm<1>, grid, dim3(256), 0, st, d, g);
  hipLaunchKernelGGL(k_exp_gemm<2>, grid, dim3(256), 0, st, d, g);
  hipLaunchKernelGGL(k_exp_gemm<3>, grid, dim3(256), 0, st, d, g);
  hipLaunchKernelGGL(k_exp_gemm<4>, grid, dim3(256), 0, st, d, g);
  hipLaunchKernelGGL(k_exp_gemm<5>, grid, dim3(256), 0, st, d, g);
  hipLaunchKernelGGL(k_exp_solve, dim3(d.nrhs), dim3(256), exp_solve_lds(m), st, d, g);
  return hipGetLastError();
}

hipError_t exp_set_attributes() {
  return hipFuncSetAttribute((const void*)k_exp_solve, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)((size_t)LDSM * LDSM * 8));
}

}  // namespace fab
