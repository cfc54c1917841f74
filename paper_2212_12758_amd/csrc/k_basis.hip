// Streaming kernels of the k-truncated basis construction (Algorithm 2 of the
// paper) with the sketch Theta (Section 2.1.1) fused into the pass that
// writes each new basis vector.
//
// One step i (1 <= i <= m) builds column i-1 of the Hessenberg matrix and the
// basis vector u_i with two passes over the rows:
//
//   k_dots   : w~ = A u_{i-1} (stencil or CSR), window dots d_j = u_j^T w~ for
//              j in [max(0,i-k), i-1] and ||w~||^2, written as per-block partials.
//              The last block to finish reduces the partials in a fixed order
//              (plus the norm partials of u_{i-1} from the previous update
//              pass) and writes h_{j,i-1} = d_j / (eta_j eta_{i-1}), the
//              subdiagonal entry h_{i-1,i-2} = eta_{i-1}, and the update
//              coefficients.  Extra blocks appended to the grid reduce the
//              sketch partials of column i-1.
//   k_update : u_i = w~/eta_{i-1} - sum_j (h_{j,i-1}/eta_j) u_j  (classical
//              Gram-Schmidt against the window, which equals the printed
//              modified Gram-Schmidt in exact arithmetic because the window
//              is orthonormal), stored in the basis precision; ||u_i||^2 and
//              Theta u_i are accumulated from the stored (rounded) values.
//
// Vectors are kept unnormalised (v_j = u_j / eta_j); every scale is applied
// to scalars, never by an extra pass over the vectors.  All arithmetic on
// vector elements is FP64 whatever the storage type.
#include "fab_dev.h"

namespace fab {

template <typename T>
__device__ inline double stencil_apply(const SolveDev& d, const T* __restrict__ u, int r, long long e) {
  const int nr = d.nrhs;
  const int x = r % d.nx;
  const int yz = r / d.nx;
  const int y = yz % d.ny;
  const int z = yz / d.ny;
  double w = d.c[0] * (double)u[e];
  if (x > 0) w += d.c[1] * (double)u[e - nr];
  if (x < d.nx - 1) w += d.c[2] * (double)u[e + nr];
  const long long sy = (long long)d.nx * nr;
  if (y > 0) w += d.c[3] * (double)u[e - sy];
  if (y < d.ny - 1) w += d.c[4] * (double)u[e + sy];
  if (d.nz > 1) {
    const long long sz = sy * d.ny;
    if (z > 0) w += d.c[5] * (double)u[e - sz];
    if (z < d.nz - 1) w += d.c[6] * (double)u[e + sz];
  }
  return w;
}

template <typename T>
__device__ inline double csr_apply(const SolveDev& d, const T* __restrict__ u, int r, int q) {
  const int p0 = d.rowptr[r], p1 = d.rowptr[r + 1];
  double w = 0.0;
  for (int p = p0; p < p1; ++p) w += (double)d.val[p] * (double)u[(long long)d.col[p] * d.nrhs + q];
  return w;
}

__device__ inline double wave_sum_all(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline int* rhs_mused(const SolveDev& d, int q) { return d.status + 4 + 2 * q; }
__device__ inline int* rhs_brk(const SolveDev& d, int q) { return d.status + 5 + 2 * q; }

// ------------------------------------------------------------------ pass 1
// i in 1..m: dots for column i-1.  i == m+1 with nstream == 0: finishing pass
// (norm of u_m, subdiagonal h_{m+1,m}, sketch column m).
template <typename T, int OP>
__global__ void __launch_bounds__(BLOCK) k_dots(SolveDev d, int i, int nstream) {
  if (d.status[0]) return;  // every rhs has broken down already
  __shared__ double red[BLOCK / 64][NSLOT * 32];
  __shared__ unsigned ticket;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nr = d.nrhs;
  const int j0 = i - d.k > 0 ? i - d.k : 0;
  const int nw = i - j0;
  const T* __restrict__ V = (const T*)d.V;

  if ((int)blockIdx.x < nstream) {
    const int q = tid & (nr - 1);
    double acc[NSLOT];
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl) acc[sl] = 0.0;
    const T* __restrict__ src = V + (long long)(i - 1) * d.ldv;
    const long long tile_elems = (long long)d.rows_per_tile * nr;
    const long long nel = (long long)d.n * nr;
    for (int t = blockIdx.x; t < d.ntiles; t += d.nblk) {
      const long long e0 = (long long)t * tile_elems;
      const long long e1 = e0 + tile_elems < nel ? e0 + tile_elems : nel;
      for (long long e = e0 + tid; e < e1; e += BLOCK) {
        const int r = (int)(e >> d.lognrhs);
        double w;
        if (OP == OP_STENCIL) {
          w = stencil_apply(d, src, r, e);
        } else {
          w = csr_apply(d, src, r, q);
          d.wbuf[e] = w;
        }
#pragma unroll
        for (int jj = 0; jj < KMAX; ++jj)
          if (jj < nw) acc[jj] += (double)V[(long long)(j0 + jj) * d.ldv + e] * w;
        acc[KMAX] += w * w;
      }
    }
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl) {
      const double v = wave_sum_rhs(acc[sl], nr);
      if (lane < nr) red[wv][sl * nr + lane] = v;
    }
    __syncthreads();
    for (int x = tid; x < NSLOT * nr; x += BLOCK) {
      const double v = ((red[0][x] + red[1][x]) + red[2][x]) + red[3][x];
      const int sl = x / nr, qq = x - sl * nr;
      d.part[((long long)blockIdx.x * nr + qq) * NSLOT + sl] = v;
    }
  } else {
    // reduce the sketch partials of column i-1: one wave per (row, rhs)
    const int nwaves = (gridDim.x - nstream) * (BLOCK / 64);
    const int wid = (blockIdx.x - nstream) * (BLOCK / 64) + wv;
    const int col = i - 1;
    for (int rho = wid; rho < d.s * nr; rho += nwaves) {
      double v = 0.0;
      const double* p = d.skpart + (long long)rho * d.nblk;
      for (int b = lane; b < d.nblk; b += 64) v += p[b];
      v = wave_sum_all(v);
      if (lane == 0) {
        const int pr = rho >> d.lognrhs, qq = rho & (nr - 1);
        d.S[(long long)qq * d.s * (d.m + 1) + (long long)col * d.s + pr] = v * d.sk_scale;
      }
    }
  }

  // ---- last block: scalar reduction in a fixed order
  __threadfence();
  __syncthreads();
  if (tid == 0) ticket = atomicAdd(d.counter, 1u);
  __syncthreads();
  if (ticket != gridDim.x - 1) return;
  __threadfence();

  const int m = d.m;
  for (int qq = wv; qq < nr; qq += BLOCK / 64) {
    double nn = 0.0;
    for (int b = lane; b < d.nblk; b += 64) nn += d.npart[(long long)b * nr + qq];
    nn = wave_sum_all(nn);
    double sums[NSLOT];
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl) {
      double v = 0.0;
      if (nstream > 0)
        for (int b = lane; b < nstream; b += 64) v += d.part[((long long)b * nr + qq) * NSLOT + sl];
      sums[sl] = wave_sum_all(v);
    }
    if (lane == 0) {
      double* eta = d.eta + (long long)qq * (m + 1);
      double* H = d.H + (long long)qq * (m + 1) * m;
      double* wn = d.wnorm + (long long)qq * (m + 1);
      double* cf = d.coef + (long long)qq * NSLOT;
      int* mused = rhs_mused(d, qq);
      int* brk = rhs_brk(d, qq);
      const double eta_prev = sqrt(nn);  // ||u_{i-1}||
      eta[i - 1] = eta_prev;
      if (!*brk) {
        if (!isfinite(eta_prev)) {
          d.status[1] = 1;
          *brk = 1;
          *mused = i - 1;
        } else if (i == 1) {
          if (eta_prev == 0.0) { *brk = 1; *mused = 0; }
        } else if (eta_prev <= 100.0 * d.unit_round * wn[i - 2]) {
          *brk = 1;  // invariant subspace of dimension i-1
          *mused = i - 1;
          H[(long long)(i - 2) * (m + 1) + (i - 1)] = 0.0;
        } else {
          H[(long long)(i - 2) * (m + 1) + (i - 1)] = eta_prev;
        }
      }
      if (*brk || nstream == 0) {
#pragma unroll
        for (int sl = 0; sl < NSLOT; ++sl) cf[sl] = 0.0;
        if (!*brk) *mused = m;
      } else {
        wn[i - 1] = sqrt(sums[KMAX]) / eta_prev;
        cf[0] = 1.0 / eta_prev;
#pragma unroll
        for (int jj = 0; jj < KMAX; ++jj) {
          if (jj < nw) {
            const double ej = eta[j0 + jj];
            const double h = sums[jj] / (ej * eta_prev);
            H[(long long)(i - 1) * (m + 1) + (j0 + jj)] = h;
            cf[1 + jj] = h / ej;
          } else {
            cf[1 + jj] = 0.0;
          }
        }
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    int all = 1;
    for (int qq = 0; qq < nr; ++qq) all &= *rhs_brk(d, qq);
    d.status[0] = all;
    *d.counter = 0u;
  }
}

// ------------------------------------------------------------------ pass 2
// START: u_0 = fl(b).  Otherwise u_i = cf0 * w~ - sum_j cf_{1+j} u_{j0+j}.
template <typename T, int OP, int SK, bool START>
__global__ void __launch_bounds__(BLOCK) k_update(SolveDev d, int i) {
  if (d.status[0]) return;
  extern __shared__ double lds[];
  __shared__ double nred[BLOCK / 64][32];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nr = d.nrhs;
  const int q = tid & (nr - 1);
  const int R = d.rows_per_tile;
  const int tile_elems = R * nr;
  const long long nel = (long long)d.n * nr;
  const int j0 = i - d.k > 0 ? i - d.k : 0;
  const int nw = START ? 0 : i - j0;
  T* __restrict__ V = (T*)d.V;
  const T* __restrict__ src = START ? nullptr : V + (long long)(i - 1) * d.ldv;
  T* __restrict__ dst = V + (long long)i * d.ldv;

  double cw = 1.0;
  double cj[KMAX];
  {
    const double* cf = d.coef + (long long)q * NSLOT;
    if (!START) cw = cf[0];
#pragma unroll
    for (int jj = 0; jj < KMAX; ++jj) cj[jj] = START ? 0.0 : cf[1 + jj];
  }

  double* X = lds;                                        // SRHT tile [R][nr]
  double* acc = lds + (SK == SK_SRHT ? tile_elems : 0);   // sketch accumulator [s][nr]
  const int snr = d.s * nr;
  for (int x = tid; x < snr; x += BLOCK) acc[x] = 0.0;
  __syncthreads();

  double nrm = 0.0;
  for (int t = blockIdx.x; t < d.ntiles; t += d.nblk) {
    const long long e0 = (long long)t * tile_elems;
    for (int l = tid; l < tile_elems; l += BLOCK) {
      const long long e = e0 + l;
      double uu = 0.0;
      int r = (int)(e >> d.lognrhs);
      if (e < nel) {
        double u;
        if (START) {
          u = d.b[e];
        } else {
          double w;
          if (OP == OP_STENCIL) w = stencil_apply(d, src, r, e);
          else w = d.wbuf[e];
          u = cw * w;
#pragma unroll
          for (int jj = 0; jj < KMAX; ++jj)
            if (jj < nw) u -= cj[jj] * (double)V[(long long)(j0 + jj) * d.ldv + e];
        }
        const T ut = (T)u;
        dst[e] = ut;
        uu = (double)ut;
        nrm += uu * uu;
        if (SK == SK_SPARSE) {
          int rows[ZMAX];
          unsigned long long sb;
          sparse_sign_column(d.key_a, d.key_b, r, d.s, d.zeta, rows, &sb);
#pragma unroll
          for (int tt = 0; tt < ZMAX; ++tt)
            if (tt < d.zeta) atomicAdd(&acc[rows[tt] * nr + q], ((sb >> tt) & 1ull) ? -uu : uu);
        }
      }
      if (SK == SK_SRHT) {
        const double sgn = (sm64_out(d.key_a, (unsigned long long)r) >> 63) ? -1.0 : 1.0;
        X[l] = uu * sgn;
      }
    }
    if (SK == SK_SRHT) {
      __syncthreads();
      // Walsh-Hadamard transform of the tile along rows (Sylvester order).
      for (int h = 1; h < R; h <<= 1) {
        for (int bi = tid; bi < (R >> 1) * nr; bi += BLOCK) {
          const int qq = bi & (nr - 1);
          const int pr = bi >> d.lognrhs;
          const int lo = ((pr & ~(h - 1)) << 1) | (pr & (h - 1));
          const int a = lo * nr + qq, bb = (lo + h) * nr + qq;
          const double xa = X[a], xb = X[bb];
          X[a] = xa + xb;
          X[bb] = xa - xb;
        }
        __syncthreads();
      }
      // sampled rows r = (r_hi, r_lo): contribution (-1)^popcount(r_hi & t) * X[r_lo]
      for (int pq = tid; pq < snr; pq += BLOCK) {
        const int p = pq >> d.lognrhs, qq = pq & (nr - 1);
        const int rr = d.srht_rows[p];
        const int par = __popc((unsigned)(rr >> d.log_rows) & (unsigned)t) & 1;
        const double v = X[(rr & (R - 1)) * nr + qq];
        acc[pq] += par ? -v : v;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int pq = tid; pq < snr; pq += BLOCK) d.skpart[(long long)pq * d.nblk + blockIdx.x] = acc[pq];

  nrm = wave_sum_rhs(nrm, nr);
  if (lane < nr) nred[wv][lane] = nrm;
  __syncthreads();
  if (tid < nr)
    d.npart[(long long)blockIdx.x * nr + tid] = ((nred[0][tid] + nred[1][tid]) + nred[2][tid]) + nred[3][tid];
}

// ------------------------------------------------------------------ combine
// out = sum_j cf_j u_j with cf_j = beta c_j / eta_j (FP64 accumulation).
template <typename T>
__global__ void __launch_bounds__(BLOCK) k_combine(SolveDev d, const double* __restrict__ cf, int mmax,
                                                   double* __restrict__ out) {
  const T* __restrict__ V = (const T*)d.V;
  const long long nel = (long long)d.n * d.nrhs;
  const int nr = d.nrhs;
  for (long long e = (long long)blockIdx.x * BLOCK + threadIdx.x; e < nel; e += (long long)gridDim.x * BLOCK) {
    const int q = (int)(e & (nr - 1));
    const double* c = cf + (long long)q * (d.m + 1);
    double a = 0.0;
    for (int j = 0; j < mmax; ++j) a += c[j] * (double)V[(long long)j * d.ldv + e];
    out[e] = a;
  }
}

// ------------------------------------------------------------------ host launchers
template <typename T>
static hipError_t launch_dots_t(const SolveDev& d, int i, hipStream_t st) {
  if (d.op == OP_STENCIL)
    hipLaunchKernelGGL((k_dots<T, OP_STENCIL>), dim3(d.nblk + d.nred), dim3(BLOCK), 0, st, d, i, d.nblk);
  else
    hipLaunchKernelGGL((k_dots<T, OP_CSR>), dim3(d.nblk + d.nred), dim3(BLOCK), 0, st, d, i, d.nblk);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_update_t(const SolveDev& d, int i, hipStream_t st, size_t lds_update) {
  if (d.op == OP_STENCIL) {
    if (d.sketch == SK_SRHT)
      hipLaunchKernelGGL((k_update<T, OP_STENCIL, SK_SRHT, false>), dim3(d.nblk), dim3(BLOCK), lds_update, st, d, i);
    else
      hipLaunchKernelGGL((k_update<T, OP_STENCIL, SK_SPARSE, false>), dim3(d.nblk), dim3(BLOCK), lds_update, st, d, i);
  } else {
    if (d.sketch == SK_SRHT)
      hipLaunchKernelGGL((k_update<T, OP_CSR, SK_SRHT, false>), dim3(d.nblk), dim3(BLOCK), lds_update, st, d, i);
    else
      hipLaunchKernelGGL((k_update<T, OP_CSR, SK_SPARSE, false>), dim3(d.nblk), dim3(BLOCK), lds_update, st, d, i);
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_start_t(const SolveDev& d, hipStream_t st, size_t lds_update) {
  if (d.sketch == SK_SRHT)
    hipLaunchKernelGGL((k_update<T, OP_STENCIL, SK_SRHT, true>), dim3(d.nblk), dim3(BLOCK), lds_update, st, d, 0);
  else
    hipLaunchKernelGGL((k_update<T, OP_STENCIL, SK_SPARSE, true>), dim3(d.nblk), dim3(BLOCK), lds_update, st, d, 0);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_finish_t(const SolveDev& d, hipStream_t st) {
  hipLaunchKernelGGL((k_dots<T, OP_STENCIL>), dim3(d.nred), dim3(BLOCK), 0, st, d, d.m + 1, 0);
  return hipGetLastError();
}

template <typename T>
static hipError_t set_lds_attr() {
  const int mx = 160 * 1024;
  hipError_t e = hipSuccess;
  auto f = [&](const void* k) { hipError_t r = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, mx); if (r != hipSuccess) e = r; };
  f((const void*)k_update<T, OP_STENCIL, SK_SRHT, false>);
  f((const void*)k_update<T, OP_STENCIL, SK_SPARSE, false>);
  f((const void*)k_update<T, OP_CSR, SK_SRHT, false>);
  f((const void*)k_update<T, OP_CSR, SK_SPARSE, false>);
  f((const void*)k_update<T, OP_STENCIL, SK_SRHT, true>);
  f((const void*)k_update<T, OP_STENCIL, SK_SPARSE, true>);
  return e;
}

hipError_t basis_set_attributes() {
  hipError_t e = set_lds_attr<float>();
  if (e != hipSuccess) return e;
  return set_lds_attr<double>();
}

hipError_t basis_start(const SolveDev& d, int esize, hipStream_t st, size_t lds) {
  return esize == 4 ? launch_start_t<float>(d, st, lds) : launch_start_t<double>(d, st, lds);
}
hipError_t basis_dots(const SolveDev& d, int esize, int i, hipStream_t st) {
  return esize == 4 ? launch_dots_t<float>(d, i, st) : launch_dots_t<double>(d, i, st);
}
hipError_t basis_update(const SolveDev& d, int esize, int i, hipStream_t st, size_t lds) {
  return esize == 4 ? launch_update_t<float>(d, i, st, lds) : launch_update_t<double>(d, i, st, lds);
}
hipError_t basis_finish(const SolveDev& d, int esize, hipStream_t st) {
  return esize == 4 ? launch_finish_t<float>(d, st) : launch_finish_t<double>(d, st);
}
hipError_t basis_combine(const SolveDev& d, int esize, const double* cf, int mmax, double* out, hipStream_t st) {
  const long long nel = (long long)d.n * d.nrhs;
  long long g = (nel + BLOCK - 1) / BLOCK;
  if (g > 8192) g = 8192;
  if (esize == 4) hipLaunchKernelGGL(k_combine<float>, dim3((unsigned)g), dim3(BLOCK), 0, st, d, cf, mmax, out);
  else hipLaunchKernelGGL(k_combine<double>, dim3((unsigned)g), dim3(BLOCK), 0, st, d, cf, mmax, out);
  return hipGetLastError();
}

}  // namespace fab

namespace fab {

__global__ void k_zero(unsigned long long* p, long long n8) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n8; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// bytes must be a multiple of 8 (workspace regions are 256-byte aligned).
hipError_t zero_fill(void* p, size_t bytes, hipStream_t st) {
  const long long n8 = (long long)(bytes / 8);
  if (n8 == 0) return hipSuccess;
  long long g = (n8 + 255) / 256;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)g), dim3(256), 0, st, (unsigned long long*)p, n8);
  return hipGetLastError();
}

// SRHT row sampling, one wave: Floyd's algorithm draws s distinct rows of
// [0, npad): for t = 0..s-1 with j = npad - s + t, q = floor(u_t (j+1) / 2^64)
// (u_t the t-th output of the row stream); q is taken unless already
// present, else j.  Lanes test membership in parallel.
__global__ void __launch_bounds__(64) k_srht_rows(int* rows, long long npad, int s, unsigned long long key) {
  const int lane = threadIdx.x;
  for (int t = 0; t < s; ++t) {
    const unsigned long long j = (unsigned long long)(npad - s + t);
    const unsigned long long v = sm64_out(key, (unsigned long long)t);
    const long long qv = (long long)__umul64hi(v, j + 1ull);
    bool hit = false;
    for (int u = lane; u < t; u += 64) hit |= (rows[u] == (int)qv);
    const unsigned long long any = __ballot(hit);
    if (lane == 0) rows[t] = any ? (int)j : (int)qv;
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
  }
}

hipError_t srht_sample_rows(int* rows, long long npad, int s, unsigned long long key, hipStream_t st) {
  hipLaunchKernelGGL(k_srht_rows, dim3(1), dim3(64), 0, st, rows, npad, s, key);
  return hipGetLastError();
}

}  // namespace fab
