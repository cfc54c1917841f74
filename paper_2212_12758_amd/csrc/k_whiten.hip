// Whitening of the truncated basis (Section 2.1.2): the sketch Theta V_i of
// the basis built by Algorithm 2 is monitored, and once its condition
// exceeds a threshold the basis is replaced by V_i R^{-1} (Theta V_i = Q R),
// the Hessenberg matrix by R Hbar_{i-1} R_{i-1}^{-1} and the sketch by Q;
// later steps follow Algorithm 1 (k_bg.hip).
//
//   k_wh_col    after the update pass of step i, one workgroup per rhs adds
//               column a = i-1 to the triangular factor R of the normalised
//               sketch (Theta v_j = S[:, j] / eta_j) and to X = R^{-1}:
//                 g = (Theta V_{a+1})^T Theta v_a,  R[:a, a] = X^T g[:a],
//                 R[a, a] = sqrt(g_a - ||R[:a, a]||^2),
//                 X[:a, a] = -X R[:a, a] / R[a, a],  X[a, a] = 1 / R[a, a],
//               and keeps the largest column sums of |R| and |X|, whose
//               product is kappa_1(R) = ||R||_1 ||R^{-1}||_1.  On a check step
//               it raises the flag when kappa_1(R) exceeds the threshold (or
//               the factorisation broke down).
//   k_wh_prod,  many workgroups (one output per thread): Hbar_{i-1} <-
//   k_wh_fin    R_i Hbar_{i-1} X_{i-1} (column i-1 of H, left by the
//               discarded step i, is cleared), the sketch S[:, j] <-
//               (Theta V_i X)[:, j] (j >= 1), the scales eta_0 <- eta_0 R_00
//               (the stored u_0 = b is kept) and eta_j <- 1, and the
//               coefficients C[l, j] = X[l, j] / eta_l of the basis
//               transform; k_wh_prod forms T = Hbar X, the rescaled sketch
//               and C, k_wh_fin the products with R and the copies.
//   k_wh_basis  u_j <- sum_{l <= j} C[l, j] u_l for 1 <= j < i, in place
//               (each thread owns one element of every vector; output
//               columns are produced in descending blocks so that no input is
//               overwritten before it is read); k_wh_basis1, for one rhs,
//               stages the coefficients in LDS.
//
// Per-rhs scratch in the dense workspace (region oM, ld m): R at 0, X at m^2,
// products at 2m^2 and 3m^2, C at 4m^2, scalars at 5m^2; the rescaled sketch
// is staged in region oW.
#include "k_basis.h"

namespace fab {

namespace {

constexpr int WB = 256;     // threads per workgroup
constexpr int WH_MAXS = 8192;
enum { WS_MAXR = 0, WS_MAXX = 1, WS_SING = 2, WS_KAPPA = 3 };

__device__ inline double wh_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wv = wave_id();
  v = wave_sum_all(v);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < WB / 64; ++w) t += red[w];
  return t;
}

__global__ void __launch_bounds__(WB) k_wh_col(SolveDev d, DenseDev g, int a, int check, double thresh,
                                               int* flag, int cj) {
  extern __shared__ double sa[];     // Theta v_a (s values), then cj staged columns of S
  __shared__ double gsh[512], rsh[512];
  __shared__ double red[WB / 64];
  const int q = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = wave_id();
  if (d.status[5 + 2 * q]) return;   // broken down: nothing to monitor
  const int m = d.m, m1 = m + 1, s = d.s;
  const long long mm = (long long)m * m;
  double* ws = g.base + (long long)q * g.stride + g.oM;
  double* R = ws;
  double* X = ws + mm;
  double* sc = ws + 5 * mm;
  const double* S = d.S + (long long)q * s * m1;
  const double* eta = d.eta + (long long)q * m1;
  const double ea = eta[a];
  for (int r = tid; r < s; r += WB) sa[r] = S[(long long)a * s + r] / ea;
  __syncthreads();
  // g_l = (Theta v_l)^T Theta v_a, l <= a: four columns per wave at a time,
  // the columns staged in LDS in chunks of cj (eight loads in flight)
  double* ch = sa + s;
  for (int lc = 0; lc <= a; lc += cj) {
    const int cn = a + 1 - lc < cj ? a + 1 - lc : cj;
    __syncthreads();   // sa written / the previous chunk's dots are done
    const double* src = S + (long long)lc * s;
    const long long n2 = (long long)cn * s;
    long long x = tid;
    for (; x + 7 * WB < n2; x += 8 * WB) {
      double t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = src[x + u * WB];
#pragma unroll
      for (int u = 0; u < 8; ++u) ch[x + u * WB] = t[u];
    }
    for (; x < n2; x += WB) ch[x] = src[x];
    __syncthreads();
    for (int l0 = 4 * wv; l0 < cn; l0 += 4 * (WB / 64)) {
      double t[4] = {0.0, 0.0, 0.0, 0.0};
      for (int r = lane; r < s; r += 64) {
        const double xv = sa[r];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (l0 + u < cn) t[u] += ch[(long long)(l0 + u) * s + r] * xv;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double tu = wave_sum_all(t[u]);
        const int l = lc + l0 + u;
        if (lane == 0 && l0 + u < cn) gsh[l] = tu / eta[l];
      }
    }
  }
  __syncthreads();
  // R[:a, a] = X^T g (X upper triangular: column l has rows 0..l)
  double p2 = 0.0;
  for (int l = tid; l < a; l += WB) {
    double t = 0.0;
#pragma unroll 8
    for (int u = 0; u <= l; ++u) t += X[u + (long long)l * m] * gsh[u];
    rsh[l] = t;
    R[l + (long long)a * m] = t;
    p2 += t * t;
  }
  const double rr = gsh[a] - wh_sum(p2, red);   // the sum's barriers publish rsh
  const bool sing = !(rr > 0.0) || !isfinite(rr);
  const double raa = sing ? 0.0 : sqrt(rr);
  // X[:a, a] = -X[:a, :a] R[:a, a] / R[a, a]
  double cx = 0.0, cr = 0.0;
  for (int t0 = tid; t0 < a; t0 += WB) {
    double v = 0.0;
#pragma unroll 8
    for (int l = t0; l < a; ++l) v += X[t0 + (long long)l * m] * rsh[l];
    const double xv = sing ? 0.0 : -v / raa;
    X[t0 + (long long)a * m] = xv;
    cx += fabs(xv);
    cr += fabs(rsh[t0]);
  }
  cx = wh_sum(cx, red);
  cr = wh_sum(cr, red);
  if (tid == 0) {
    R[a + (long long)a * m] = raa;
    X[a + (long long)a * m] = sing ? 0.0 : 1.0 / raa;
    const double colR = cr + raa, colX = cx + (sing ? 0.0 : 1.0 / raa);
    const double mr = a == 0 ? colR : fmax(sc[WS_MAXR], colR);
    const double mx = a == 0 ? colX : fmax(sc[WS_MAXX], colX);
    const double sg = (a == 0 ? 0.0 : sc[WS_SING]) + (sing ? 1.0 : 0.0);
    sc[WS_MAXR] = mr;
    sc[WS_MAXX] = mx;
    sc[WS_SING] = sg;
    sc[WS_KAPPA] = sg != 0.0 ? INFINITY : mr * mx;
    if (check && (sg != 0.0 || mr * mx > thresh)) *flag = 1;
  }
}

// The products of the whitening transform, spread over many workgroups (one
// output per thread, each summed in the same order as a single workgroup
// would): T = Hbar_{i-1} X_{i-1} (i x (i-1), ld m), the rescaled sketch
// Sw[:, j] = sum_{l <= j} (S[:, l] / eta_l) X[l, j] (s x i) and the basis
// coefficients C[l, j] = X[l, j] / eta_l (1 <= j < i).  blockIdx.y = rhs.
__global__ void __launch_bounds__(WB) k_wh_prod(SolveDev d, DenseDev g, int i) {
  const int q = blockIdx.y;
  if (d.status[5 + 2 * q]) return;
  const int m = d.m, m1 = m + 1, s = d.s;
  const long long mm = (long long)m * m;
  double* base = g.base + (long long)q * g.stride;
  double* ws = base + g.oM;
  const double* X = ws + mm;
  double* T = ws + 2 * mm;
  double* C = ws + 4 * mm;
  double* Sw = base + g.oW;
  const double* H = d.H + (long long)q * m1 * m;
  const double* S = d.S + (long long)q * s * m1;
  const double* eta = d.eta + (long long)q * m1;
  const long long nT = (long long)i * (i - 1), nS = (long long)s * i, nC = (long long)i * i;
  for (long long x = (long long)blockIdx.x * WB + threadIdx.x; x < nT + nS + nC; x += (long long)gridDim.x * WB) {
    if (x < nT) {
      const int r = (int)(x % i), c = (int)(x / i);
      double t = 0.0;
      for (int l = 0; l <= c; ++l) t += H[r + (long long)l * m1] * X[l + (long long)c * m];
      T[r + (long long)c * m] = t;
    } else if (x < nT + nS) {
      const long long y = x - nT;
      const int r = (int)(y % s), j = (int)(y / s);
      double t = 0.0;
      for (int l = 0; l <= j; ++l) t += S[(long long)l * s + r] / eta[l] * X[l + (long long)j * m];
      Sw[r + (long long)j * s] = t;
    } else {
      const long long y = x - nT - nS;
      const int l = (int)(y % i), j = (int)(y / i);
      C[l + (long long)j * m] = (j >= 1 && l <= j) ? X[l + (long long)j * m] / eta[l] : 0.0;
    }
  }
}

// Hbar_{i-1} <- R_i T (rows 0..i-1, columns 0..i-2; column i-1 cleared), the
// sketch S[:, j] <- Sw[:, j] for 1 <= j < i (column 0 keeps Theta u_0 =
// eta'_0 q_0) and the scales eta_0 <- eta_0 R_00, eta_j <- 1.  blockIdx.y = rhs.
__global__ void __launch_bounds__(WB) k_wh_fin(SolveDev d, DenseDev g, int i) {
  const int q = blockIdx.y;
  if (d.status[5 + 2 * q]) return;
  const int m = d.m, m1 = m + 1, s = d.s;
  const long long mm = (long long)m * m;
  double* base = g.base + (long long)q * g.stride;
  double* ws = base + g.oM;
  const double* R = ws;
  const double* T = ws + 2 * mm;
  const double* Sw = base + g.oW;
  double* H = d.H + (long long)q * m1 * m;
  double* S = d.S + (long long)q * s * m1;
  double* eta = d.eta + (long long)q * m1;
  const long long nH = (long long)i * (i - 1), nS = (long long)s * i;
  for (long long x = (long long)blockIdx.x * WB + threadIdx.x; x < nH + nS + m1; x += (long long)gridDim.x * WB) {
    if (x < nH) {
      const int r = (int)(x % i), c = (int)(x / i);
      double t = 0.0;
      for (int l = r; l < i; ++l) t += R[r + (long long)l * m] * T[l + (long long)c * m];
      H[r + (long long)c * m1] = t;
    } else if (x < nH + nS) {
      const long long y = x - nH;
      if (y >= s) S[y] = Sw[y];
    } else {
      H[(x - nH - nS) + (long long)(i - 1) * m1] = 0.0;
    }
  }
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) eta[0] = eta[0] * R[0];
    for (int j = 1 + threadIdx.x; j < i; j += WB) eta[j] = 1.0;
  }
}

// In-place u_j <- sum_{l <= j} C[l, j] u_l, 1 <= j < i.
template <typename T>
__global__ void __launch_bounds__(256) k_wh_basis(SolveDev d, DenseDev g, int i) {
  constexpr int JB = 32;   // output columns per block (accumulators per thread)
  const int nr = d.nrhs, m = d.m;
  const long long nel = (long long)d.n * nr;
  T* __restrict__ V = (T*)d.V;
  const long long mm = (long long)m * m;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < nel; e += (long long)gridDim.x * 256) {
    const int q = (int)(e & (nr - 1));
    if (d.status[5 + 2 * q]) continue;
    const double* C = g.base + (long long)q * g.stride + g.oM + 4 * mm;
    const int nblk = (i - 1 + JB - 1) / JB;
    for (int bj = nblk - 1; bj >= 0; --bj) {
      const int j0 = 1 + bj * JB, j1 = j0 + JB < i ? j0 + JB : i;   // outputs [j0, j1)
      double acc[JB];
#pragma unroll
      for (int u = 0; u < JB; ++u) acc[u] = 0.0;
      for (int l = 0; l < j1; ++l) {
        const double x = (double)V[(long long)l * d.ldv + e];
#pragma unroll
        for (int u = 0; u < JB; ++u) {
          const int j = j0 + u;
          if (j < j1 && l <= j) acc[u] += C[l + (long long)j * m] * x;
        }
      }
#pragma unroll
      for (int u = 0; u < JB; ++u)
        if (j0 + u < j1) V[(long long)(j0 + u) * d.ldv + e] = (T)acc[u];
    }
  }
}

// One right-hand side: the same transform with the coefficients of each
// group of WJB output columns staged in LDS (Cs[l][u] = C[l, j0+u], zero
// where l > j), two consecutive elements per thread (one 8- or 16-byte load
// per input column) and WJB outputs accumulated per element, so the basis is
// read ceil((i-1)/WJB) times in total per group instead of once per group of
// a single element's registers, and every coefficient read is an LDS
// broadcast.  Groups go from the last columns down, so a group only reads
// columns that no earlier group has overwritten.
constexpr int WJB = 32;
template <typename T>
__global__ void __launch_bounds__(256) k_wh_basis1(SolveDev d, DenseDev g, int i) {
  extern __shared__ double Cs[];   // [i][WJB]
  if (d.status[5]) return;         // the rhs broke down
  const int m = d.m;
  const long long n = d.n;
  T* __restrict__ V = (T*)d.V;
  const double* C = g.base + g.oM + 4 * (long long)m * m;
  const long long e = ((long long)blockIdx.x * 256 + threadIdx.x) * 2;
  const bool pair = e + 1 < n;
  const int nb = (i - 1 + WJB - 1) / WJB;
  for (int bj = nb - 1; bj >= 0; --bj) {
    const int j0 = 1 + bj * WJB, j1 = j0 + WJB < i ? j0 + WJB : i;   // outputs [j0, j1)
    __syncthreads();
    for (int x = threadIdx.x; x < j1 * WJB; x += 256) {
      const int l = x / WJB, j = j0 + x % WJB;
      Cs[x] = (j < j1 && l <= j) ? C[l + (long long)j * m] : 0.0;
    }
    __syncthreads();
    if (e >= n) continue;
    double a0[WJB], a1[WJB];
#pragma unroll
    for (int u = 0; u < WJB; ++u) a0[u] = a1[u] = 0.0;
#pragma unroll 2
    for (int l = 0; l < j1; ++l) {
      const T* src = V + (long long)l * d.ldv + e;
      double x0, x1 = 0.0;
      if (pair) {
        if constexpr (sizeof(T) == 4) {
          const float2 v = *reinterpret_cast<const float2*>(src);
          x0 = v.x;
          x1 = v.y;
        } else {
          const double2 v = *reinterpret_cast<const double2*>(src);
          x0 = v.x;
          x1 = v.y;
        }
      } else {
        x0 = (double)src[0];
      }
      const double* cl = Cs + l * WJB;
#pragma unroll
      for (int u = 0; u < WJB; ++u) {
        a0[u] += cl[u] * x0;
        a1[u] += cl[u] * x1;
      }
    }
#pragma unroll
    for (int u = 0; u < WJB; ++u) {
      if (j0 + u < j1) {
        T* dst = V + (long long)(j0 + u) * d.ldv + e;
        dst[0] = (T)a0[u];
        if (pair) dst[1] = (T)a1[u];
      }
    }
  }
}

}  // namespace

// Column a = i-1 of the incremental factor; check != 0 tests the threshold.
hipError_t wh_col(const SolveDev& d, const DenseDev& g, int a, int check, double thresh, int* flag,
                  hipStream_t st) {
  if (d.s > WH_MAXS || d.m + 1 > 512) return hipErrorInvalidValue;
  // columns of S staged in LDS beside Theta v_a: as many as fit in 150 KB
  long long cj = ((long long)(150 * 1024 / 8) - d.s) / d.s;
  if (cj < 1) return hipErrorInvalidValue;
  if (cj > a + 1) cj = a + 1;
  hipLaunchKernelGGL(k_wh_col, dim3(d.nrhs), dim3(WB), (size_t)(1 + cj) * d.s * 8, st, d, g, a, check, thresh, flag,
                     (int)cj);
  return hipGetLastError();
}

hipError_t wh_whiten(const SolveDev& d, const DenseDev& g, int esize, int i, hipStream_t st) {
  {
    const long long work = (long long)d.s * i + 2LL * i * i;
    long long gb = (work + WB - 1) / WB;
    if (gb > 1024) gb = 1024;
    hipLaunchKernelGGL(k_wh_prod, dim3((unsigned)gb, d.nrhs), dim3(WB), 0, st, d, g, i);
    hipLaunchKernelGGL(k_wh_fin, dim3((unsigned)gb, d.nrhs), dim3(WB), 0, st, d, g, i);
  }
  if (d.nrhs == 1) {
    const long long gr = ((long long)d.n + 511) / 512;
    const size_t lds = (size_t)i * WJB * 8;
    if (gr > 0x7fffffffLL || lds > 160 * 1024) return hipErrorInvalidValue;
    if (esize == 4) hipLaunchKernelGGL(k_wh_basis1<float>, dim3((unsigned)gr), dim3(256), lds, st, d, g, i);
    else hipLaunchKernelGGL(k_wh_basis1<double>, dim3((unsigned)gr), dim3(256), lds, st, d, g, i);
    return hipGetLastError();
  }
  const long long nel = (long long)d.n * d.nrhs;
  long long gr = (nel + 255) / 256;
  if (gr > 8192) gr = 8192;
  if (esize == 4) hipLaunchKernelGGL(k_wh_basis<float>, dim3((unsigned)gr), dim3(256), 0, st, d, g, i);
  else hipLaunchKernelGGL(k_wh_basis<double>, dim3((unsigned)gr), dim3(256), 0, st, d, g, i);
  return hipGetLastError();
}

hipError_t wh_set_attributes() {
  hipError_t e = hipFuncSetAttribute((const void*)k_wh_col, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
  hipError_t r;
  if ((r = hipFuncSetAttribute((const void*)k_wh_basis1<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               160 * 1024)) != hipSuccess)
    e = r;
  if ((r = hipFuncSetAttribute((const void*)k_wh_basis1<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               160 * 1024)) != hipSuccess)
    e = r;
  return e;
}

}  // namespace fab
