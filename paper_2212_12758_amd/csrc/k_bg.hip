// Basis built by orthogonalising a sketch (Algorithm 1 of the paper, the
// construction of Section 2.1.1 due to Balabanov & Grigori): the sketch
// S_i = Theta V_i is kept orthonormal by one classical Gram-Schmidt step per
// column on s-vectors, and the same coefficients act on the long vectors.
//
// Step i (1 <= i <= m) with the stored vectors u_j (v_j = u_j / eta_j):
//
//   k_bg_apply  : w~ = A u_{i-1} in FP64 and the per-block partials of
//                 Theta w~ (CSR operators keep w~ for the update pass).
//   k_bg_reduce : fixed-order reduction of those partials into S[:, i].
//   k_bg_gs     : one workgroup per right-hand side: p = S[:, i] / eta_{i-1}
//                 (= Theta A v_{i-1}), r_j = s_j^T p for j < i, the sketch
//                 residual p - S_{i-1} r (optionally a second pass on it),
//                 r_ii = its norm, the breakdown test
//                 r_ii <= 100 u ||p||, the Hessenberg column (r; r_ii), and
//                 the update weights 1/eta_{i-1} and r_j / eta_j.
//   k_bg_update : u_i = w~ / eta_{i-1} - sum_{j<i} (r_j / eta_j) u_j, so that
//                 v_i = u_i / r_ii with eta_i = r_ii and Theta u_i = the sketch
//                 residual (stored as S[:, i]).
//
// The first vector is u_0 = fl(b) (written with its sketch partials by the
// start pass of the truncated basis); k_bg_gs at i = 0 sets eta_0 = r_11 =
// ||Theta b||.  The result is r_11 V_m f(H_hat) e_1 as for the truncated
// basis, so the dense tail, the least-squares refinement and the combination
// are shared.
#include "k_basis.h"

namespace fab {

namespace {

constexpr int GS_BLOCK = 256;
constexpr int GS_MAXS = 8192;
constexpr size_t GS_LDS_MAX = 150 * 1024;
// Dynamic LDS of the Gram-Schmidt step: p (s values), plus the sketch columns
// S[:, 0..m-1] when they fit (every access of the step is then an LDS access).
size_t gs_lds_staged(int s, int m) { return (size_t)s * (m + 1) * 8; }
bool gs_staged(int s, int m) { return gs_lds_staged(s, m) <= GS_LDS_MAX; }

// ------------------------------------------------------------------ pass 1
template <typename T, int OP, int SK, int LT>
__global__ void __launch_bounds__(1 << (LT - 3)) k_bg_apply(SolveDev d, int i) {
  constexpr int BLOCK = 1 << (LT - 3);
  constexpr int NW = BLOCK / 64;
  constexpr int TILE = 1 << LT;
  extern __shared__ double lds[];
  const int tid = threadIdx.x, wv = wave_id();
  const int nr = d.nrhs;
  const long long nel = (long long)d.n * nr;
  const T* __restrict__ src = (const T*)d.V + (long long)(i - 1) * d.ldv;
  double* X = lds;                                          // SRHT tile (padded)
  double* acc = lds + (SK == SK_SRHT ? padx(TILE) : 0);     // sketch accumulator [s][nr]
  const int snr = d.s * nr;
  // sparse sign: one accumulator per wave when LDS was sized for it (fixed order)
  const int nsl = (SK == SK_SPARSE && NW > 1 && d.sk_slices == NW) ? NW : 1;
  double* acc_w = acc + (nsl > 1 ? wv * snr : 0);
  int* rows_l = (int*)(acc + snr * nsl);
  for (int x = tid; x < snr * nsl; x += BLOCK) acc[x] = 0.0;
  if (SK == SK_SRHT)
    for (int x = tid; x < d.s; x += BLOCK) rows_l[x] = d.srht_rows[x];
  __syncthreads();
  const TileWalk tw = tile_walk(d, blockIdx.x);
  for (int u = tw.u0; u < tw.uhi; u += tw.step) {
    const int t = walk_tile(d, tw, u);
    const long long e = ((long long)t << LT) + (long long)tid * EPT;
    double w[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) w[j] = 0.0;
    if (e < nel) {
      if constexpr (OP == OP_STENCIL) {
        double c[EPT];
        get8(src, e, nel, c);
        apply8<T>(d, src, e, nel, c, w);
        // the stencil also yields values for padding rows past n: not part of w~
#pragma unroll
        for (int j = 0; j < EPT; ++j)
          if (e + j >= nel) w[j] = 0.0;
      } else {
        get8(d.wbuf, e, nel, w);   // w~ from the CSR product pass (zero past n)
      }
      if (SK == SK_SPARSE) {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          if (e + j < nel) {
            const int r = (int)((e + j) >> d.lognrhs);
            const int q = (int)((e + j) & (nr - 1));
            int rows[ZMAX];
            unsigned long long sb;
            sparse_sign_column(d.key_a, d.key_b, r, d.s, d.zeta, rows, &sb);
#pragma unroll
            for (int tt = 0; tt < ZMAX; ++tt)
              if (tt < d.zeta) atomicAdd(&acc_w[rows[tt] * nr + q], ((sb >> tt) & 1ull) ? -w[j] : w[j]);
          }
        }
      }
    }
    if (SK == SK_SRHT) {
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const unsigned long long r = (unsigned long long)((e + j) >> d.lognrhs);
        if (sm64_out(d.key_a, r) >> 63) w[j] = -w[j];
      }
      fwht_tile<LT>(w, X, d.lognrhs);
      for (int pq = tid; pq < snr; pq += BLOCK) {
        const int p = pq >> d.lognrhs, qq = pq & (nr - 1);
        const int rr = rows_l[p];
        const int par = __popc((unsigned)(rr >> d.log_rows) & (unsigned)t) & 1;
        const double v = X[padx(((rr & (d.rows_per_tile - 1)) << d.lognrhs) + qq)];
        acc[pq] += par ? -v : v;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  double* skp = d.skpart + (long long)(i & 1) * d.skstride;
  for (int pq = tid; pq < snr; pq += BLOCK) {
    double a = acc[pq];
    for (int sl = 1; sl < nsl; ++sl) a += acc[sl * snr + pq];
    skp[((long long)(pq >> 3) * d.nblk + blockIdx.x) * 8 + (pq & 7)] = a;
  }
}

__global__ void __launch_bounds__(256) k_bg_reduce(SolveDev d, int col) {
  reduce_sketch_column<256>(d, col, blockIdx.x, gridDim.x);
}

// Fixed-order sum over the workgroup; every thread gets the result.
__device__ inline double gs_block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wv = wave_id();
  v = wave_sum_all(v);
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < GS_BLOCK / 64; ++w) t += red[w];
  return t;
}

// ------------------------------------------------------------------ small Gram-Schmidt on the sketch
// cf: [nrhs][m+2] update weights (cf[0] = 1/eta_{i-1}, cf[1+j] = r_j/eta_j).
// passes = 2 repeats the step on its own residual and adds the coefficients
// (r = r' + r''), which keeps S orthonormal to rounding when one classical
// pass does not; the long vectors still see one update with the total r.
template <bool STAGED>
__global__ void __launch_bounds__(GS_BLOCK) k_bg_gs(SolveDev d, double* __restrict__ cfall, int i, int passes,
                                                    int cj) {
  // p, then the residual (s values); staged: S[:, 0..i-1] behind it;
  // chunked (!STAGED, cj > 0): the residual, then cj columns of S
  extern __shared__ double psh[];
  __shared__ double csh[512];          // r_j / eta_j
  __shared__ double cnew[512];         // this pass's coefficients
  __shared__ double red[GS_BLOCK / 64];
  const int q = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = wave_id();
  const int m = d.m, m1 = d.m + 1, s = d.s;
  double* S = d.S + (long long)q * s * m1;
  double* eta = d.eta + (long long)q * m1;
  double* H = d.H + (long long)q * m1 * m;
  double* cf = cfall + (long long)q * (m + 2);
  if (*rhs_brk(d, q)) {
    for (int x = tid; x <= i; x += GS_BLOCK) cf[x] = 0.0;
    return;
  }
  if (i == 0) {
    double a = 0.0;
    for (int r = tid; r < s; r += GS_BLOCK) a += S[r] * S[r];
    const double r11 = sqrt(gs_block_sum(a, red));
    if (tid == 0) {
      if (!isfinite(r11)) {
        d.status[1] = 1;
        *rhs_brk(d, q) = 1;
        *rhs_mused(d, q) = 0;
      } else if (r11 == 0.0) {
        *rhs_brk(d, q) = 1;
        *rhs_mused(d, q) = 0;
      } else {
        eta[0] = r11;
      }
    }
    return;
  }
  const double eprev = eta[i - 1];
  double* Si = S + (long long)i * s;
  double a = 0.0;
  for (int r = tid; r < s; r += GS_BLOCK) {
    const double v = Si[r] / eprev;
    psh[r] = v;
    a += v * v;
  }
  // columns 0..i-1: their LDS copy (STAGED, a compile-time choice so that
  // the accesses compile to LDS loads) or global memory
  if (STAGED) {
    // eight loads in flight per thread
    const long long n2 = (long long)i * s;
    long long x = tid;
    for (; x + 7 * GS_BLOCK < n2; x += 8 * GS_BLOCK) {
      double t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = S[x + u * GS_BLOCK];
#pragma unroll
      for (int u = 0; u < 8; ++u) psh[s + x + u * GS_BLOCK] = t[u];
    }
    for (; x < n2; x += GS_BLOCK) psh[s + x] = S[x];
  }
  const double* Sc = STAGED ? (const double*)(psh + s) : (const double*)S;
  const double pn = sqrt(gs_block_sum(a, red));   // includes the barrier after psh (and Sl) is written
  for (int j = tid; j < i; j += GS_BLOCK) csh[j] = 0.0;
  double rii = 0.0;
  if (!STAGED && cj > 0) {
    // S too large for LDS: columns visited in chunks of cj staged in LDS.
    // The dots of a chunk use the pass's vector x (psh, unchanged during the
    // pass) and its terms are subtracted from the residual res at once, so
    // one sweep over S serves both halves of the classical Gram-Schmidt
    // step, in the same order of operations as the unchunked loops.
    double* res = psh + s;
    double* ch = psh + 2 * s;
    for (int pass = 0; pass < passes; ++pass) {
      for (int r = tid; r < s; r += GS_BLOCK) res[r] = psh[r];
      for (int jc = 0; jc < i; jc += cj) {
        const int cn = i - jc < cj ? i - jc : cj;
        __syncthreads();   // the previous chunk's residual is done with ch
        const double* src = S + (long long)jc * s;
        const long long n2 = (long long)cn * s;
        long long x = tid;
        for (; x + 7 * GS_BLOCK < n2; x += 8 * GS_BLOCK) {
          double t[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) t[u] = src[x + u * GS_BLOCK];
#pragma unroll
          for (int u = 0; u < 8; ++u) ch[x + u * GS_BLOCK] = t[u];
        }
        for (; x < n2; x += GS_BLOCK) ch[x] = src[x];
        __syncthreads();
        for (int j0 = 4 * wv; j0 < cn; j0 += 4 * (GS_BLOCK / 64)) {
          double t[4] = {0.0, 0.0, 0.0, 0.0};
          for (int r = lane; r < s; r += 64) {
            const double xv = psh[r];
#pragma unroll
            for (int u = 0; u < 4; ++u)
              if (j0 + u < cn) t[u] += ch[(long long)(j0 + u) * s + r] * xv;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const double tu = wave_sum_all(t[u]);
            const int j = jc + j0 + u;
            if (lane == 0 && j0 + u < cn) cnew[j] = tu / (eta[j] * eta[j]);
          }
        }
        __syncthreads();
        for (int r = tid; r < s; r += GS_BLOCK) {
          double v = res[r];
#pragma unroll 8
          for (int j = 0; j < cn; ++j) v -= cnew[jc + j] * ch[(long long)j * s + r];
          res[r] = v;
        }
      }
      __syncthreads();
      double b2 = 0.0;
      for (int r = tid; r < s; r += GS_BLOCK) {
        const double v = res[r];
        psh[r] = v;
        b2 += v * v;
      }
      for (int j = tid; j < i; j += GS_BLOCK) csh[j] += cnew[j];
      rii = sqrt(gs_block_sum(b2, red));   // barriers: psh, csh complete before the next pass
    }
  } else {
    for (int pass = 0; pass < passes; ++pass) {
      // coefficients s_j^T x of the current vector x (p, then the residual),
      // s_j = S[:, j] / eta_j: one wave per column, stored as r_j / eta_j
      // (four columns per wave at a time, so that their loads overlap)
      for (int j0 = 4 * wv; j0 < i; j0 += 4 * (GS_BLOCK / 64)) {
        double t[4] = {0.0, 0.0, 0.0, 0.0};
        for (int r = lane; r < s; r += 64) {
          const double x = psh[r];
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (j0 + u < i) t[u] += Sc[(long long)(j0 + u) * s + r] * x;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double tu = wave_sum_all(t[u]);
          if (lane == 0 && j0 + u < i) cnew[j0 + u] = tu / (eta[j0 + u] * eta[j0 + u]);
        }
      }
      __syncthreads();
      // residual x - sum_j r_j s_j (each thread its own rows)
      double b2 = 0.0;
      for (int r = tid; r < s; r += GS_BLOCK) {
        double v = psh[r];
#pragma unroll 8
        for (int j = 0; j < i; ++j) v -= cnew[j] * Sc[(long long)j * s + r];
        psh[r] = v;
        b2 += v * v;
      }
      for (int j = tid; j < i; j += GS_BLOCK) csh[j] += cnew[j];
      rii = sqrt(gs_block_sum(b2, red));   // barriers: psh, csh complete before the next pass
    }
  }
  for (int r = tid; r < s; r += GS_BLOCK) Si[r] = psh[r];   // Theta u_i
  const bool nonfinite = !isfinite(pn) || !isfinite(rii);
  const bool brk = nonfinite || rii <= 100.0 * d.unit_round * pn;
  for (int j = tid; j < i; j += GS_BLOCK) {
    H[(long long)(i - 1) * m1 + j] = csh[j] * eta[j];
    cf[1 + j] = brk ? 0.0 : csh[j];
  }
  if (tid == 0) {
    cf[0] = brk ? 0.0 : 1.0 / eprev;
    if (nonfinite) {
      d.status[1] = 1;
      *rhs_brk(d, q) = 1;
      *rhs_mused(d, q) = i - 1;
    } else if (brk) {
      *rhs_brk(d, q) = 1;            // span{v_0..v_{i-1}} is invariant
      *rhs_mused(d, q) = i;
    } else {
      H[(long long)(i - 1) * m1 + i] = rii;
      eta[i] = rii;
      if (i == m) *rhs_mused(d, q) = m;
    }
  }
}

// ------------------------------------------------------------------ pass 2: u_i = cf0 w~ - V_{i-1} (cf_1..cf_i)
template <typename T, int OP, bool NR1>
__global__ void __launch_bounds__(256) k_bg_update(SolveDev d, const double* __restrict__ cf, int i) {
  const int nr = d.nrhs;
  const long long nel = (long long)d.n * nr;
  const long long cld = d.m + 2;
  T* __restrict__ V = (T*)d.V;
  const T* __restrict__ src = V + (long long)(i - 1) * d.ldv;
  T* __restrict__ dst = V + (long long)i * d.ldv;
  for (long long e = ((long long)blockIdx.x * 256 + threadIdx.x) * EPT; e < nel;
       e += (long long)gridDim.x * 256 * EPT) {
    double w[EPT], a[EPT];
    if (OP == OP_STENCIL) {
      double c[EPT];
      get8(src, e, nel, c);
      stencil8(d, src, e, nel, c, w);
    } else {
      get8(d.wbuf, e, nel, w);
    }
    long long cb[EPT];   // start of each element's weights
#pragma unroll
    for (int j = 0; j < EPT; ++j) cb[j] = NR1 ? 0 : (long long)((e + j) & (nr - 1)) * cld;
#pragma unroll
    for (int j = 0; j < EPT; ++j) a[j] = cf[cb[j]] * w[j];
    if (e + EPT <= nel) {
      int jv = 0;
      for (; jv + 4 <= i; jv += 4) {
        double v[4][EPT];
#pragma unroll
        for (int u = 0; u < 4; ++u) load8(V + (long long)(jv + u) * d.ldv + e, v[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int j = 0; j < EPT; ++j) a[j] -= cf[cb[j] + 1 + jv + u] * v[u][j];
      }
      for (; jv < i; ++jv) {
        double v[EPT];
        load8(V + (long long)jv * d.ldv + e, v);
#pragma unroll
        for (int j = 0; j < EPT; ++j) a[j] -= cf[cb[j] + 1 + jv] * v[j];
      }
      double rounded[EPT];
      store8(dst + e, a, rounded);
    } else {
      for (int jv = 0; jv < i; ++jv) {
        double v[EPT];
        get8(V + (long long)jv * d.ldv, e, nel, v);
#pragma unroll
        for (int j = 0; j < EPT; ++j) a[j] -= cf[cb[j] + 1 + jv] * v[j];
      }
      for (int j = 0; j < EPT; ++j)
        if (e + j < nel) dst[e + j] = (T)a[j];
    }
  }
}

template <typename T, int OP>
hipError_t apply_t(const SolveDev& d, int i, hipStream_t st, size_t lds) {
  const dim3 g(d.nblk);
  if (OP == OP_CSR) {
    const hipError_t r = operator_product(d, (const T*)d.V + (long long)(i - 1) * d.ldv, (int)sizeof(T), d.wbuf, st);
    if (r != hipSuccess) return r;
  }
  if (d.log_tile == 11) {
    if (d.sketch == SK_SRHT) hipLaunchKernelGGL((k_bg_apply<T, OP, SK_SRHT, 11>), g, dim3(256), lds, st, d, i);
    else hipLaunchKernelGGL((k_bg_apply<T, OP, SK_SPARSE, 11>), g, dim3(256), lds, st, d, i);
  } else {
    if (d.sketch == SK_SRHT) hipLaunchKernelGGL((k_bg_apply<T, OP, SK_SRHT, 9>), g, dim3(64), lds, st, d, i);
    else hipLaunchKernelGGL((k_bg_apply<T, OP, SK_SPARSE, 9>), g, dim3(64), lds, st, d, i);
  }
  return hipGetLastError();
}

template <typename T, int OP>
hipError_t update_t(const SolveDev& d, const double* cf, int i, hipStream_t st) {
  const long long nel = (long long)d.n * d.nrhs;
  long long g = (nel + 256 * EPT - 1) / (256 * EPT);
  if (g > 4096) g = 4096;
  if (d.nrhs == 1) hipLaunchKernelGGL((k_bg_update<T, OP, true>), dim3((unsigned)g), dim3(256), 0, st, d, cf, i);
  else hipLaunchKernelGGL((k_bg_update<T, OP, false>), dim3((unsigned)g), dim3(256), 0, st, d, cf, i);
  return hipGetLastError();
}

template <typename T, int OP>
void attr_t(hipError_t& e) {
  auto f = [&](const void* k) {
    const hipError_t r = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (r != hipSuccess) e = r;
  };
  f((const void*)k_bg_apply<T, OP, SK_SRHT, 11>);
  f((const void*)k_bg_apply<T, OP, SK_SPARSE, 11>);
  f((const void*)k_bg_apply<T, OP, SK_SRHT, 9>);
  f((const void*)k_bg_apply<T, OP, SK_SPARSE, 9>);
}

}  // namespace

hipError_t bg_apply(const SolveDev& d, int esize, int i, hipStream_t st, size_t lds) {
  const bool csr = d.op == OP_CSR;
  if (esize == 4) return csr ? apply_t<float, OP_CSR>(d, i, st, lds) : apply_t<float, OP_STENCIL>(d, i, st, lds);
  return csr ? apply_t<double, OP_CSR>(d, i, st, lds) : apply_t<double, OP_STENCIL>(d, i, st, lds);
}

hipError_t bg_reduce(const SolveDev& d, int col, hipStream_t st) {
  hipLaunchKernelGGL(k_bg_reduce, dim3(d.nred), dim3(256), 0, st, d, col);
  return hipGetLastError();
}

// i = 0: r_11 = ||Theta b||; i >= 1: the Gram-Schmidt step of column i
// (passes = 1 as in Algorithm 1, 2 with the step repeated).
hipError_t bg_gs(const SolveDev& d, double* cf, int i, int passes, hipStream_t st) {
  if (d.s > GS_MAXS || d.m + 1 > 512 || passes < 1 || passes > 2) return hipErrorInvalidValue;
  if (gs_staged(d.s, d.m)) {
    hipLaunchKernelGGL(k_bg_gs<true>, dim3(d.nrhs), dim3(GS_BLOCK), gs_lds_staged(d.s, d.m), st, d, cf, i, passes, 0);
  } else {
    // columns in LDS chunks when at least 4 fit beside p and the residual
    const long long cj = ((long long)(GS_LDS_MAX / 8) - 2LL * d.s) / d.s;
    if (cj >= 4)
      hipLaunchKernelGGL(k_bg_gs<false>, dim3(d.nrhs), dim3(GS_BLOCK), (size_t)(2 + cj) * d.s * 8, st, d, cf, i,
                         passes, (int)cj);
    else
      hipLaunchKernelGGL(k_bg_gs<false>, dim3(d.nrhs), dim3(GS_BLOCK), (size_t)d.s * 8, st, d, cf, i, passes, 0);
  }
  return hipGetLastError();
}

hipError_t bg_update(const SolveDev& d, int esize, const double* cf, int i, hipStream_t st) {
  const bool csr = d.op == OP_CSR;
  if (esize == 4) return csr ? update_t<float, OP_CSR>(d, cf, i, st) : update_t<float, OP_STENCIL>(d, cf, i, st);
  return csr ? update_t<double, OP_CSR>(d, cf, i, st) : update_t<double, OP_STENCIL>(d, cf, i, st);
}

hipError_t bg_set_attributes() {
  hipError_t e = hipSuccess;
  attr_t<float, OP_STENCIL>(e);
  attr_t<float, OP_CSR>(e);
  attr_t<double, OP_STENCIL>(e);
  attr_t<double, OP_CSR>(e);
  hipError_t r = hipFuncSetAttribute((const void*)k_bg_gs<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)GS_LDS_MAX);
  if (r != hipSuccess) e = r;
  r = hipFuncSetAttribute((const void*)k_bg_gs<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(GS_MAXS * 8 > (int)GS_LDS_MAX ? GS_MAXS * 8 : (int)GS_LDS_MAX));
  if (r != hipSuccess) e = r;
  return e;
}

}  // namespace fab
