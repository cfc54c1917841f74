// Streaming kernels of the k-truncated basis construction (Algorithm 2 of the
// paper) with the sketch Theta (Section 2.1.1) fused into the pass that
// writes each new basis vector.
//
// One step i (1 <= i <= m) builds column i-1 of the Hessenberg matrix and the
// basis vector u_i with two passes over the rows:
//
//   k_dots   : w~ = A u_{i-1} (stencil; a CSR operator's w~ comes from
//              the product kernel launched just before), window dots d_j = u_j^T w~ for
//              j in [max(0,i-k), i-1] and ||w~||^2, written as per-block
//              partials (a pure streaming pass).
//   k_update : every streaming block first reduces those partials, in a fixed
//              order, together with the norm partials of u_{i-1} from the
//              previous update pass, and derives eta_{i-1}, the breakdown
//              test, h_{j,i-1} = d_j / (eta_j eta_{i-1}) and the update
//              coefficients (block 0 publishes them).  Extra blocks appended
//              to the grid reduce the sketch partials of column i-1.  Then
//              u_i = w~/eta_{i-1} - sum_j (h_{j,i-1}/eta_j) u_j  (classical
//              Gram-Schmidt against the window, which equals the printed
//              modified Gram-Schmidt in exact arithmetic because the window
//              is orthonormal), stored in the basis precision; ||u_i||^2 and
//              Theta u_i are accumulated from the stored (rounded) values.
//
// Vectors are kept unnormalised (v_j = u_j / eta_j); every scale is applied
// to scalars, never by an extra pass over the vectors.  All arithmetic on
// vector elements is FP64 whatever the storage type.
//
// Work layout: tiles of TILE = 2^LT consecutive elements (rows x rhs); a
// block of TILE/8 threads owns one tile at a time and each thread owns 8
// consecutive elements, moved with 16-byte vector loads and stores.  Basis
// columns start on 256-byte boundaries.  QC = 1 when there is one right-hand
// side (one accumulator per quantity); QC = 8 otherwise (one per element).
#pragma once
#include "fab_dev.h"

namespace fab {

constexpr int EPT = 8;   // elements per thread per tile

// y = A x for the CSR operator (k_csr.hip); x is FP32 (esize 4) or FP64.
hipError_t csr_spmv(const SolveDev& d, const void* x, int esize, double* y, hipStream_t st);
// w~ = A x (d.prod == PROD_CSR) or A (A x) (PROD_SQ_*) into y (k_csr.hip).
hipError_t operator_product(const SolveDev& d, const void* x, int esize, double* y, hipStream_t st);

// ------------------------------------------------------------------ 8-element memory helpers
__device__ inline void load8(const float* __restrict__ p, double* v) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}
__device__ inline void load8(const double* __restrict__ p, double* v) {
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const double2 a = *reinterpret_cast<const double2*>(p + 2 * h);
    v[2 * h] = a.x;
    v[2 * h + 1] = a.y;
  }
}
__device__ inline void store8(float* __restrict__ p, const double* v, double* rounded) {
  float4 a, b;
  a.x = (float)v[0]; a.y = (float)v[1]; a.z = (float)v[2]; a.w = (float)v[3];
  b.x = (float)v[4]; b.y = (float)v[5]; b.z = (float)v[6]; b.w = (float)v[7];
  *reinterpret_cast<float4*>(p) = a;
  *reinterpret_cast<float4*>(p + 4) = b;
  rounded[0] = a.x; rounded[1] = a.y; rounded[2] = a.z; rounded[3] = a.w;
  rounded[4] = b.x; rounded[5] = b.y; rounded[6] = b.z; rounded[7] = b.w;
}
__device__ inline void store8(double* __restrict__ p, const double* v, double* rounded) {
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    double2 a;
    a.x = v[2 * h];
    a.y = v[2 * h + 1];
    *reinterpret_cast<double2*>(p + 2 * h) = a;
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) rounded[j] = v[j];
}
// 8 consecutive elements kept in the storage type until they are used (FP32
// values take one register each instead of two).
__device__ inline void load8r(const float* __restrict__ p, float* v) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 4);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
}
__device__ inline void load8r(const double* __restrict__ p, double* v) { load8(p, v); }
template <typename T>
__device__ inline double ldg1(const T* __restrict__ u, long long x, long long nel) {
  return (x >= 0 && x < nel) ? (double)u[x] : 0.0;
}
template <typename T>
constexpr int vec_align() { return 16 / (int)sizeof(T); }

// u[e+off .. e+off+7]: vector load when aligned and in range, else guarded scalars.
template <typename T>
__device__ inline void fetch8(const T* __restrict__ u, long long e, long long off, long long nel, double* v) {
  const long long a = e + off;
  if ((off % vec_align<T>()) == 0 && a >= 0 && a + EPT <= nel) {
    load8(u + a, v);
  } else {
#pragma unroll
    for (int j = 0; j < EPT; ++j) v[j] = ldg1(u, a + j, nel);
  }
}

template <typename T>
__device__ inline void get8(const T* __restrict__ p, long long e, long long nel, double* v) {
  if (e + EPT <= nel) {
    load8(p + e, v);
  } else {
#pragma unroll
    for (int j = 0; j < EPT; ++j) v[j] = ldg1(p, e + j, nel);
  }
}

// Boundary masks of elements e..e+7 (row = element >> lognrhs): bit j of
// mx0 is set when element j has an x-1 neighbour, mx1 for x+1, etc.
struct Masks8 {
  unsigned mx0, mx1, my0, my1, mz0, mz1;
};
__device__ inline Masks8 masks8(const SolveDev& d, long long e) {
  const int r0 = (int)(e >> d.lognrhs);
  int x = r0 % d.nx;
  const int yz = r0 / d.nx;
  int y = yz % d.ny;
  int z = yz / d.ny;
  int rp = r0;
  Masks8 mk{0u, 0u, 0u, 0u, 0u, 0u};
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int r = (int)((e + j) >> d.lognrhs);
    if (r != rp) {
      rp = r;
      if (++x == d.nx) {
        x = 0;
        if (++y == d.ny) { y = 0; ++z; }
      }
    }
    mk.mx0 |= (unsigned)(x > 0) << j;
    mk.mx1 |= (unsigned)(x < d.nx - 1) << j;
    mk.my0 |= (unsigned)(y > 0) << j;
    mk.my1 |= (unsigned)(y < d.ny - 1) << j;
    mk.mz0 |= (unsigned)(z > 0) << j;
    mk.mz1 |= (unsigned)(z < d.nz - 1) << j;
  }
  return mk;
}

// Values at e+j-S (DIR < 0) or e+j+S (DIR > 0), j = 0..7, for a shift S < 8
// known at compile time: inside the group they are centre values.
template <typename T, int S, int DIR>
__device__ inline void shifted8(const T* __restrict__ u, long long e, long long nel, const double* c, double* nb) {
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int src = j + DIR * S;
    nb[j] = (src >= 0 && src < EPT) ? c[src >= 0 && src < EPT ? src : 0] : ldg1(u, e + src, nel);
  }
}

template <typename T, int DIR>
__device__ inline void xneighbour8(const T* __restrict__ u, long long e, long long nel, int nr, const double* c,
                                   double* nb) {
  if (nr == 1) shifted8<T, 1, DIR>(u, e, nel, c, nb);
  else if (nr == 2) shifted8<T, 2, DIR>(u, e, nel, c, nb);
  else if (nr == 4) shifted8<T, 4, DIR>(u, e, nel, c, nb);
  else fetch8(u, e, (long long)DIR * nr, nel, nb);
}

// w = A u at elements e..e+7 for the stencil operator; c holds u[e..e+7].
template <typename T>
__device__ inline void stencil8(const SolveDev& d, const T* __restrict__ u, long long e, long long nel,
                                const double* c, double* w) {
  const Masks8 mk = masks8(d, e);
  const int nr = d.nrhs;
  double nb[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) w[j] = d.c[0] * c[j];
  xneighbour8<T, -1>(u, e, nel, nr, c, nb);
#pragma unroll
  for (int j = 0; j < EPT; ++j) w[j] += d.c[1] * (((mk.mx0 >> j) & 1u) ? nb[j] : 0.0);
  xneighbour8<T, 1>(u, e, nel, nr, c, nb);
#pragma unroll
  for (int j = 0; j < EPT; ++j) w[j] += d.c[2] * (((mk.mx1 >> j) & 1u) ? nb[j] : 0.0);
  const long long sy = (long long)d.nx * nr;
  fetch8(u, e, -sy, nel, nb);
#pragma unroll
  for (int j = 0; j < EPT; ++j) w[j] += d.c[3] * (((mk.my0 >> j) & 1u) ? nb[j] : 0.0);
  fetch8(u, e, sy, nel, nb);
#pragma unroll
  for (int j = 0; j < EPT; ++j) w[j] += d.c[4] * (((mk.my1 >> j) & 1u) ? nb[j] : 0.0);
  if (d.nz > 1) {
    const long long sz = sy * d.ny;
    fetch8(u, e, -sz, nel, nb);
#pragma unroll
    for (int j = 0; j < EPT; ++j) w[j] += d.c[5] * (((mk.mz0 >> j) & 1u) ? nb[j] : 0.0);
    fetch8(u, e, sz, nel, nb);
#pragma unroll
    for (int j = 0; j < EPT; ++j) w[j] += d.c[6] * (((mk.mz1 >> j) & 1u) ? nb[j] : 0.0);
  }
}

// Branch-free w = A u at e..e+7 when the y stride n_x*nrhs keeps vector loads
// aligned and nrhs is 1 or a multiple of 8: every load is issued
// unconditionally and the boundary conditions are applied to the values, so
// the loads of a tile overlap.  Neighbour addresses are clamped into
// [0, nel); a clamped value is always masked out when the 8 elements share
// their grid row (n_x a multiple of 8, or nrhs >= 8), otherwise the caller
// restricts this path to tiles whose neighbourhood lies inside [0, nel)
// (stencil_reach).  In 2D the z offsets are 0 (the centre again, masked out).
template <typename T>
__device__ inline void stencil8_fast(const SolveDev& d, const T* __restrict__ u, long long e, const double* c,
                                     double* w) {
  const Masks8 mk = masks8(d, e);
  const int nr = d.nrhs;
  const long long sy = (long long)d.nx * nr, sz = d.nz > 1 ? sy * d.ny : 0;
  double xm[EPT], xp[EPT], ym[EPT], yp[EPT], zm[EPT], zp[EPT];
  const long long nel = (long long)d.n * nr;
  load8(u + (e >= sy ? e - sy : e), ym);
  load8(u + (e + sy + EPT <= nel ? e + sy : e), yp);
  load8(u + (e >= sz ? e - sz : e), zm);
  load8(u + (e + sz + EPT <= nel ? e + sz : e), zp);
  if (nr == 1) {
    const double l = (double)u[e >= 1 ? e - 1 : e];
    const double r = (double)u[e + EPT < nel ? e + EPT : e];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      xm[j] = j == 0 ? l : c[j > 0 ? j - 1 : 0];
      xp[j] = j == EPT - 1 ? r : c[j < EPT - 1 ? j + 1 : 0];
    }
  } else {
    load8(u + (e >= nr ? e - nr : e), xm);
    load8(u + (e + nr + EPT <= nel ? e + nr : e), xp);
  }
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    double a = d.c[0] * c[j];
    a += d.c[1] * (((mk.mx0 >> j) & 1u) ? xm[j] : 0.0);
    a += d.c[2] * (((mk.mx1 >> j) & 1u) ? xp[j] : 0.0);
    a += d.c[3] * (((mk.my0 >> j) & 1u) ? ym[j] : 0.0);
    a += d.c[4] * (((mk.my1 >> j) & 1u) ? yp[j] : 0.0);
    a += d.c[5] * (((mk.mz0 >> j) & 1u) ? zm[j] : 0.0);
    a += d.c[6] * (((mk.mz1 >> j) & 1u) ? zp[j] : 0.0);
    w[j] = a;
  }
}

// Grid coordinates of row r by floating-point division with an integer
// correction (exact for r < 2^31): cheaper than two integer divisions.
__device__ inline void row_xyz(const SolveDev& d, int r, int& x, int& y, int& z) {
  int q = (int)((double)r / (double)d.nx);
  if (q * d.nx > r) --q;
  else if ((q + 1) * d.nx <= r) ++q;
  x = r - q * d.nx;
  int zz = (int)((double)q / (double)d.ny);
  if (zz * d.ny > q) --zz;
  else if ((zz + 1) * d.ny <= q) ++zz;
  y = q - zz * d.ny;
  z = zz;
}

// As stencil8_fast, with the loaded values kept in the storage type T until
// each is multiplied (same operations in the same order, FP64 arithmetic).
// With nrhs >= 8 the 8 elements are the right-hand sides of one grid row:
// the boundary conditions are applied once per thread to the coefficients
// (a neighbour outside the grid gets coefficient 0) instead of per element
// to the values.
template <typename T>
__device__ inline void stencil8_fast_raw(const SolveDev& d, const T* __restrict__ u, long long e, const T* c,
                                         double* w) {
  const int nr = d.nrhs;
  if (nr >= EPT) {
    int x, y, z;
    row_xyz(d, (int)(e >> d.lognrhs), x, y, z);
    const long long sy = (long long)d.nx * nr, sz = d.nz > 1 ? sy * d.ny : 0;
    const long long nel = (long long)d.n * nr;
    T xm[EPT], xp[EPT], ym[EPT], yp[EPT], zm[EPT], zp[EPT];
    load8r(u + (e >= sy ? e - sy : e), ym);
    load8r(u + (e + sy + EPT <= nel ? e + sy : e), yp);
    load8r(u + (e >= sz ? e - sz : e), zm);
    load8r(u + (e + sz + EPT <= nel ? e + sz : e), zp);
    load8r(u + (e >= nr ? e - nr : e), xm);
    load8r(u + (e + nr + EPT <= nel ? e + nr : e), xp);
    const double c1 = x > 0 ? d.c[1] : 0.0, c2 = x < d.nx - 1 ? d.c[2] : 0.0;
    const double c3 = y > 0 ? d.c[3] : 0.0, c4 = y < d.ny - 1 ? d.c[4] : 0.0;
    const double c5 = z > 0 ? d.c[5] : 0.0, c6 = z < d.nz - 1 ? d.c[6] : 0.0;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      double a = d.c[0] * (double)c[j];
      a += c1 * (double)xm[j];
      a += c2 * (double)xp[j];
      a += c3 * (double)ym[j];
      a += c4 * (double)yp[j];
      a += c5 * (double)zm[j];
      a += c6 * (double)zp[j];
      w[j] = a;
    }
    return;
  }
  const Masks8 mk = masks8(d, e);
  const long long sy = (long long)d.nx * nr, sz = d.nz > 1 ? sy * d.ny : 0;
  T xm[EPT], xp[EPT], ym[EPT], yp[EPT], zm[EPT], zp[EPT];
  const long long nel = (long long)d.n * nr;
  load8r(u + (e >= sy ? e - sy : e), ym);
  load8r(u + (e + sy + EPT <= nel ? e + sy : e), yp);
  load8r(u + (e >= sz ? e - sz : e), zm);
  load8r(u + (e + sz + EPT <= nel ? e + sz : e), zp);
  if (nr == 1) {
    const T l = u[e >= 1 ? e - 1 : e];
    const T r = u[e + EPT < nel ? e + EPT : e];
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      xm[j] = j == 0 ? l : c[j > 0 ? j - 1 : 0];
      xp[j] = j == EPT - 1 ? r : c[j < EPT - 1 ? j + 1 : 0];
    }
  } else {
    load8r(u + (e >= nr ? e - nr : e), xm);
    load8r(u + (e + nr + EPT <= nel ? e + nr : e), xp);
  }
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    double a = d.c[0] * (double)c[j];
    a += d.c[1] * (((mk.mx0 >> j) & 1u) ? (double)xm[j] : 0.0);
    a += d.c[2] * (((mk.mx1 >> j) & 1u) ? (double)xp[j] : 0.0);
    a += d.c[3] * (((mk.my0 >> j) & 1u) ? (double)ym[j] : 0.0);
    a += d.c[4] * (((mk.my1 >> j) & 1u) ? (double)yp[j] : 0.0);
    a += d.c[5] * (((mk.mz0 >> j) & 1u) ? (double)zm[j] : 0.0);
    a += d.c[6] * (((mk.mz1 >> j) & 1u) ? (double)zp[j] : 0.0);
    w[j] = a;
  }
}

template <typename T>
__device__ inline bool stencil_fast_ok(const SolveDev& d) {
  return d.op == OP_STENCIL && (d.nrhs == 1 || d.nrhs >= 8) && ((long long)d.nx * d.nrhs) % vec_align<T>() == 0;
}

// Tiles [lo, hi) with lo >= reach and hi + reach <= nel may use
// stencil8_fast: 0 when groups of 8 elements share their grid row (every
// full tile qualifies), else the largest neighbour offset.
__device__ inline long long stencil_reach(const SolveDev& d) {
  if (d.nrhs >= 8 || d.nx % EPT == 0) return 0;
  const long long sy = (long long)d.nx * d.nrhs;
  const long long sz = d.nz > 1 ? sy * d.ny : 0;
  long long r = sy > sz ? sy : sz;
  return r > d.nrhs ? r : d.nrhs;
}

// w~ = A u for 8 elements of the stencil operator (a CSR operator is applied
// by csr_spmv as a pass of its own).
template <typename T>
__device__ inline void apply8(const SolveDev& d, const T* __restrict__ src, long long e, long long nel,
                              const double* c, double* w) {
  stencil8(d, src, e, nel, c, w);
}

__device__ inline double wave_sum_all(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline int* rhs_mused(const SolveDev& d, int q) { return d.status + 4 + 2 * q; }
__device__ inline int* rhs_brk(const SolveDev& d, int q) { return d.status + 5 + 2 * q; }

// Fixed-order block-wide sums of RC values per thread; result in out[0..RC) for every thread.
template <int BLOCK, int RC>
__device__ inline void block_sums(const double* a, double* red /* [BLOCK/64][RC] */, double* out) {
  const int lane = threadIdx.x & 63, wv = wave_id();
#pragma unroll
  for (int c = 0; c < RC; ++c) {
    const double v = wave_sum_all(a[c]);
    if (lane == 0) red[wv * RC + c] = v;
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < RC; ++c) {
    double t = 0.0;
    for (int w = 0; w < BLOCK / 64; ++w) t += red[w * RC + c];
    out[c] = t;
  }
  __syncthreads();
}

// Reduce the per-block sketch partials of column `col` into S[:, col].
// Sketch partials of one column: layout [row / 8][block][row % 8] (rows =
// sketch row x rhs), so that a block stores whole 64-byte lines and a
// reducing wave loads 8 blocks x 8 rows per instruction.  One workgroup per
// group of 8 rows: its waves split the blocks, lanes (block % 8, row % 8)
// accumulate in a fixed order, then a butterfly over the block bits and a
// fixed-order sum over the waves.
template <int BLOCK>
__device__ void reduce_sketch_column(const SolveDev& d, int col, int g0, int gstride) {
  constexpr int NW = BLOCK / 64;
  __shared__ double rs_red[NW * 8];
  const int lane = threadIdx.x & 63, wv = wave_id();
  const int nr = d.nrhs;
  const int snr = d.s * nr;
  const int ngroups = (snr + 7) >> 3;
  const double* base = d.skpart + (long long)(col & 1) * d.skstride;
  const int chunk = (d.nblk + NW - 1) / NW;
  const int b_lo = wv * chunk, b_hi = b_lo + chunk < d.nblk ? b_lo + chunk : d.nblk;
  const int bsub = lane >> 3, rr = lane & 7;
  for (int g = g0; g < ngroups; g += gstride) {
    const double* p = base + (long long)g * d.nblk * 8;
    double v = 0.0;
    for (int b0 = b_lo; b0 < b_hi; b0 += 64) {
      double x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int b = b0 + 8 * u + bsub;
        x[u] = b < b_hi ? p[(long long)b * 8 + rr] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) v += x[u];
    }
    v += __shfl_xor(v, 8, 64);
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (lane < 8) rs_red[wv * 8 + lane] = v;
    __syncthreads();
    if (threadIdx.x < 8) {
      double t = 0.0;
      for (int w = 0; w < NW; ++w) t += rs_red[w * 8 + threadIdx.x];
      const int rho = g * 8 + (int)threadIdx.x;
      if (rho < snr) {
        const int pr = rho >> d.lognrhs, qq = rho & (nr - 1);
        d.S[(long long)qq * d.s * (d.m + 1) + (long long)col * d.s + pr] = t * d.sk_scale;
      }
    }
    __syncthreads();
  }
}

// element j of thread tid: accumulator slot and rhs
template <int QC>
__device__ inline int slot_of(int j) { return QC == 1 ? 0 : j; }
template <int QC>
__device__ inline int rhs_of(int tid, int j, int nr) { return QC == 1 ? 0 : ((tid * EPT + j) & (nr - 1)); }

// ------------------------------------------------------------------ pass 1
// i in 1..m: dots for column i-1.  i == m+1 with nstream == 0: finishing pass
// (norm of u_m, subdiagonal h_{m+1,m}, sketch column m).
template <typename T, int OP, int LT, int QC, int KT>
__global__ void __launch_bounds__(1 << (LT - 3)) k_dots(SolveDev d, int i, int nstream) {
  constexpr int BLOCK = 1 << (LT - 3);
  constexpr int NW = BLOCK / 64;
  constexpr int RC = 10;
  if (d.status[0]) return;  // every rhs has broken down already
  __shared__ double red[NW * RC];
  const int tid = threadIdx.x, lane = tid & 63, wv = wave_id();
  const int nr = d.nrhs;
  const int j0 = i - d.k > 0 ? i - d.k : 0;
  const int nw = i - j0;
  const T* __restrict__ V = (const T*)d.V;
  const int RS = NSLOT * nr;   // partial values per block: slot-major (sl * nr + q)

  if ((int)blockIdx.x < nstream) {
    double acc[NSLOT][QC];
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl)
#pragma unroll
      for (int c = 0; c < QC; ++c) acc[sl][c] = 0.0;
    const T* __restrict__ src = V + (long long)(i - 1) * d.ldv;
    const long long nel = (long long)d.n * nr;
    const bool fast_ok = OP == OP_STENCIL && nw == KT && stencil_fast_ok<T>(d);
    const long long reach = stencil_reach(d);
    const TileWalk tw = tile_walk(d, blockIdx.x);
    for (int iw = tw.u0; iw < tw.uhi; iw += tw.step) {
      const int t = walk_tile(d, tw, iw);
      const long long e = ((long long)t << LT) + (long long)tid * EPT;
      if (fast_ok && ((long long)t << LT) >= reach && (((long long)t + 1) << LT) + reach <= nel) {
        // interior tile, full window: all loads first, no branches; loaded
        // values stay in the storage type until used
        T c[EPT], win[KT > 1 ? KT - 1 : 1][EPT];
        double w[EPT];
        load8r(src + e, c);
#pragma unroll
        for (int jj = 0; jj < KT - 1; ++jj) load8r(V + (long long)(j0 + jj) * d.ldv + e, win[jj]);
        stencil8_fast_raw(d, src, e, c, w);
#pragma unroll
        for (int jj = 0; jj < KT - 1; ++jj)
#pragma unroll
          for (int j = 0; j < EPT; ++j) acc[jj][slot_of<QC>(j)] += (double)win[jj][j] * w[j];
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          acc[KT - 1][slot_of<QC>(j)] += (double)c[j] * w[j];
          acc[KMAX][slot_of<QC>(j)] += w[j] * w[j];
        }
        continue;
      }
      if (e >= nel) continue;
      double c[EPT], w[EPT];
      get8(src, e, nel, c);
      if constexpr (OP == OP_CSR) get8(d.wbuf, e, nel, w);   // w~ from the CSR product pass
      else apply8<T>(d, src, e, nel, c, w);
#pragma unroll
      for (int jj = 0; jj < KT; ++jj) {
        if (jj < nw) {
          double uj[EPT];
          if (jj == nw - 1) {
#pragma unroll
            for (int j = 0; j < EPT; ++j) uj[j] = c[j];
          } else {
            get8(V + (long long)(j0 + jj) * d.ldv, e, nel, uj);
          }
#pragma unroll
          for (int j = 0; j < EPT; ++j) acc[jj][slot_of<QC>(j)] += uj[j] * w[j];
        }
      }
#pragma unroll
      for (int j = 0; j < EPT; ++j) acc[KMAX][slot_of<QC>(j)] += w[j] * w[j];
    }
    // per (slot, rhs) block partials, fixed order
    __shared__ double pblk[NSLOT * 32];
    for (int q = 0; q < nr; ++q) {
      double a[RC];
#pragma unroll
      for (int sl = 0; sl < RC; ++sl) a[sl] = 0.0;
#pragma unroll
      for (int sl = 0; sl < NSLOT; ++sl)
#pragma unroll
        for (int c = 0; c < QC; ++c)
          if (rhs_of<QC>(tid, c, nr) == q) a[sl] += acc[sl][c];
      double o[RC];
      block_sums<BLOCK, RC>(a, red, o);
      if (tid < NSLOT) pblk[tid * nr + q] = o[tid];
    }
    __syncthreads();
    // column-major: the partials of one quantity are contiguous over the blocks
    for (int x = tid; x < RS; x += BLOCK) d.part[(long long)x * d.nblk + blockIdx.x] = pblk[x];
  }
}

// ------------------------------------------------------------------ step scalars
// Reduce, in a fixed order, the dot partials of pass 1 (part; when have_dots)
// and the norm partials of u_{i-1} (npb), then form for every rhs: eta_{i-1},
// the breakdown test, h_{j,i-1}, ||w_i|| and the update coefficients (into the
// shared array cfl[q*NSLOT + .]).  Every block computes identical values; the
// block with publish = true also stores the persistent state.
template <int BLOCK>
__device__ void step_scalars(const SolveDev& d, int i, bool have_dots, const double* __restrict__ npb, bool publish,
                             double* red, double* sums, double* cfl) {
  constexpr int RC = 10;
  const int tid = threadIdx.x;
  const int nr = d.nrhs;
  const int m = d.m;
  const int j0 = i - d.k > 0 ? i - d.k : 0;
  const int nw = i - j0;
  const int RS = NSLOT * nr;
  // scalar state of the rhs handled by this thread, loaded with the partials
  int brk_pre = 0;
  double wprev_pre = 0.0;
  double ej_pre[KMAX];
#pragma unroll
  for (int jj = 0; jj < KMAX; ++jj) ej_pre[jj] = 0.0;
  if (tid < nr) {
    brk_pre = *rhs_brk(d, tid);
    wprev_pre = i >= 2 ? d.wnorm[(long long)tid * (m + 1) + i - 2] : 0.0;
#pragma unroll
    for (int jj = 0; jj < KMAX; ++jj)
      if (jj < nw - 1) ej_pre[jj] = d.eta[(long long)tid * (m + 1) + j0 + jj];
  }
  // Quantity rr (dot slot sl = rr / nr of rhs rr % nr, or the norm of rhs
  // rr - RS) is summed over the blocks by one wave: lane l adds blocks
  // l, l + 64, ... in order, then a fixed butterfly over the lanes.  The
  // partials are column-major (contiguous over the blocks), so each wave has
  // all loads of four quantities in flight at once.
  const int RT = RS + nr;
  {
    constexpr int NWV = BLOCK / 64;
    constexpr int CPW = 4;
    const int lane = tid & 63, wv = wave_id();
    const int nb = d.nblk;
    for (int r0 = wv * CPW; r0 < RT; r0 += NWV * CPW) {
      double a[CPW];
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        a[c] = 0.0;
        const int rr = r0 + c;
        const double* col = nullptr;
        if (rr < RS) {
          const int sl = rr / nr;
          if (have_dots && (sl < nw || sl == KMAX)) col = d.part + (long long)rr * nb;
        } else if (rr < RT) {
          col = npb + (long long)(rr - RS) * nb;
        }
        if (col) {
#pragma unroll 8
          for (int b = lane; b < nb; b += 64) a[c] += col[b];
        }
      }
#pragma unroll
      for (int c = 0; c < CPW; ++c) {
        const double v = wave_sum_all(a[c]);
        if (lane == 0 && r0 + c < RT) sums[r0 + c] = v;
      }
    }
  }
  __syncthreads();

  for (int qq = tid; qq < nr; qq += BLOCK) {
    double* eta = d.eta + (long long)qq * (m + 1);
    double* H = d.H + (long long)qq * (m + 1) * m;
    double* wn = d.wnorm + (long long)qq * (m + 1);
    double* cf = cfl + qq * NSLOT;
    const int brk0 = brk_pre;
    const double wprev = wprev_pre;
    const double eta_prev = sqrt(sums[RS + qq]);  // ||u_{i-1}||, the newest window member
    double ej[KMAX];
#pragma unroll
    for (int jj = 0; jj < KMAX; ++jj) ej[jj] = (jj < nw - 1) ? ej_pre[jj] : eta_prev;
    int b = brk0, mu = -1, nonfinite = 0;
    double hsub = -1.0;   // value for H[i-1, i-2] when >= 0
    if (!b) {
      if (!isfinite(eta_prev)) {
        nonfinite = 1;
        b = 1;
        mu = i - 1;
      } else if (i == 1) {
        if (eta_prev == 0.0) { b = 1; mu = 0; }
      } else if (eta_prev <= 100.0 * d.unit_round * wprev) {
        b = 1;  // invariant subspace of dimension i-1
        mu = i - 1;
        hsub = 0.0;
      } else {
        hsub = eta_prev;
      }
    }
    if (b || !have_dots) {
      for (int sl = 0; sl < NSLOT; ++sl) cf[sl] = 0.0;
      if (!b) mu = m;
    } else {
      cf[0] = 1.0 / eta_prev;
#pragma unroll
      for (int jj = 0; jj < KMAX; ++jj) {
        if (jj < nw) {
          const double h = sums[jj * nr + qq] / (ej[jj] * eta_prev);
          cf[1 + jj] = h / ej[jj];
          if (publish) H[(long long)(i - 1) * (m + 1) + (j0 + jj)] = h;
        } else {
          cf[1 + jj] = 0.0;
        }
      }
    }
    if (publish) {
      eta[i - 1] = eta_prev;
      if (hsub >= 0.0) H[(long long)(i - 2) * (m + 1) + (i - 1)] = hsub;
      if (!b && have_dots) wn[i - 1] = sqrt(sums[KMAX * nr + qq]) / eta_prev;
      if (b != brk0) *rhs_brk(d, qq) = b;
      if (mu >= 0) *rhs_mused(d, qq) = mu;
      if (nonfinite) d.status[1] = 1;
    }
    cfl[32 * NSLOT + qq] = (double)b;   // breakdown flags after this step
  }
  __syncthreads();
  if (publish && tid == 0) {
    int all = 1;
    for (int qq = 0; qq < nr; ++qq) all &= (cfl[32 * NSLOT + qq] != 0.0);
    d.status[0] = all;
  }
}

// Finishing pass after the last update: eta_m, h_{m+1,m}, breakdown test of
// u_m (block 0) and the sketch of the last column (all blocks).
template <int LT>
__global__ void __launch_bounds__(1 << (LT - 3)) k_finish(SolveDev d) {
  constexpr int BLOCK = 1 << (LT - 3);
  constexpr int NW = BLOCK / 64;
  if (d.status[0]) return;
  __shared__ double red[NW * 10];
  __shared__ double sums[NSLOT * 32 + 32];
  __shared__ double cfl[33 * NSLOT + 32];
  const int i = d.m + 1;
  reduce_sketch_column<BLOCK>(d, i - 1, blockIdx.x, gridDim.x);
  if (blockIdx.x == 0) step_scalars<BLOCK>(d, i, false, d.npart + (long long)(d.m & 1) * d.nblk * d.nrhs, true, red, sums, cfl);
}

// ------------------------------------------------------------------ Walsh-Hadamard transform of a tile
// X holds the tile (padded index padx(e) = e + e/32).  On entry each thread
// holds its 8 consecutive elements in v (index bits 0..2); the transform acts
// on index bits [lnr, LT) (the row bits of the tile), in three-bit phases:
// registers hold three index bits, LDS transposes move between phases.  On
// exit the transformed tile is in X.
__device__ inline int padx(int e) { return e + (e >> 5); }

__device__ inline void butterflies_range(double* v, int pos, int lo, int hi) {
  // stages on index bits [lo, hi) while registers hold bits pos, pos+1, pos+2
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    if (pos + b >= lo && pos + b < hi) {
#pragma unroll
      for (int j = 0; j < EPT; ++j)
        if (!(j & (1 << b))) {
          const double x = v[j], y = v[j | (1 << b)];
          v[j] = x + y;
          v[j | (1 << b)] = x - y;
        }
    }
  }
}

template <int LT>
__device__ inline void fwht_tile(double* v, double* X, int lnr) {
  const int tid = threadIdx.x;
  butterflies_range(v, 0, lnr, 3);
  int cur = 0;
#pragma unroll
  for (int p = 3; p < LT; p += 3) {
    const int pos = p + 3 <= LT ? p : LT - 3;   // a last partial phase reuses done bits
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = (tid & ((1 << cur) - 1)) | (j << cur) | ((tid >> cur) << (cur + 3));
      X[padx(e)] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = (tid & ((1 << pos) - 1)) | (j << pos) | ((tid >> pos) << (pos + 3));
      v[j] = X[padx(e)];
    }
    __syncthreads();
    cur = pos;
    butterflies_range(v, pos, p > lnr ? p : lnr, p + 3 < LT ? p + 3 : LT);
  }
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int e = (tid & ((1 << cur) - 1)) | (j << cur) | ((tid >> cur) << (cur + 3));
    X[padx(e)] = v[j];
  }
  __syncthreads();
}

// As fwht_tile with two tile buffers used in turn, one barrier per exchange
// (a buffer is written again only after the barrier that follows all reads
// of it).  Returns the buffer that holds the transformed tile: XA after an
// odd number of stores, XB after an even number; the next transform starts
// with XA again, so a caller that read XA must pass a barrier first.
template <int LT>
__device__ inline double* fwht_tile2(double* v, double* XA, double* XB, int lnr) {
  const int tid = threadIdx.x;
  butterflies_range(v, 0, lnr, 3);
  int cur = 0;
  double* Xc = XA;
#pragma unroll
  for (int p = 3; p < LT; p += 3) {
    const int pos = p + 3 <= LT ? p : LT - 3;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = (tid & ((1 << cur) - 1)) | (j << cur) | ((tid >> cur) << (cur + 3));
      Xc[padx(e)] = v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = (tid & ((1 << pos) - 1)) | (j << pos) | ((tid >> pos) << (pos + 3));
      v[j] = Xc[padx(e)];
    }
    cur = pos;
    butterflies_range(v, pos, p > lnr ? p : lnr, p + 3 < LT ? p + 3 : LT);
    Xc = Xc == XA ? XB : XA;
  }
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int e = (tid & ((1 << cur) - 1)) | (j << cur) | ((tid >> cur) << (cur + 3));
    Xc[padx(e)] = v[j];
  }
  __syncthreads();
  return Xc;
}

// ------------------------------------------------------------------ pass 2
// Slot pq of the s x nrhs SRHT accumulators belongs to thread pq mod BLOCK
// for the whole launch.  With one rhs (at most srht_reg_slots * BLOCK slots)
// a thread keeps its slots in registers, so the per-tile sums need no LDS
// read-modify-write; otherwise the slots live in LDS and each thread updates
// its own in batches of SK_BATCH (all loads of a batch before its stores).
// The host sets d.sk_reg when the register variant applies.
template <int QC>
constexpr int srht_reg_slots() { return QC == 1 ? 4 : 0; }
constexpr int SK_BATCH = 8;


// Update coefficient `slot` (0: of w~, 1 + j: of window vector j) of the rhs
// of element j of this thread.  One rhs: uniform registers; several: read
// from the block's coefficient table in LDS at the point of use, which keeps
// 8 x NSLOT values per thread out of the registers.
template <int QC>
struct UpdCoef {
  double c1[NSLOT];   // QC == 1
  const double* tab;  // QC == 8: cfl
  __device__ inline double get(int tid, int j, int nr, int slot) const {
    if constexpr (QC == 1) return c1[slot];
    else return tab[rhs_of<QC>(tid, j, nr) * NSLOT + slot];
  }
};

// START: u_0 = fl(b).  Otherwise u_i = cf0 * w~ - sum_j cf_{1+j} u_{j0+j}.
template <typename T, int OP, int SK, bool START, int LT, int QC, int KT>
__global__ void __launch_bounds__(1 << (LT - 3)) k_update(SolveDev d, int i) {
  constexpr int BLOCK = 1 << (LT - 3);
  constexpr int TILE = 1 << LT;
  constexpr int NW = BLOCK / 64;
  constexpr int RA = (SK == SK_SRHT && srht_reg_slots<QC>() > 0) ? srht_reg_slots<QC>() : 1;
  if (d.status[0]) return;
  extern __shared__ double lds[];
  __shared__ double nred[NW][32];
  // leading blocks reduce the sketch partials of column i-1 (written by the
  // previous update pass into the other buffer)
  const int nlead = START ? 0 : d.nred;
  if ((int)blockIdx.x < nlead) {
    reduce_sketch_column<BLOCK>(d, i - 1, blockIdx.x, nlead);
    return;
  }
  const int blk = blockIdx.x - nlead;
  __shared__ double sred[NW * 10];
  __shared__ double ssums[NSLOT * 32 + 32];
  __shared__ double cfl[33 * NSLOT + 32];
  if (!START) {
    step_scalars<BLOCK>(d, i, true, d.npart + (long long)((i - 1) & 1) * d.nblk * d.nrhs, blk == 0, sred, ssums, cfl);
  }
  const int tid = threadIdx.x, lane = tid & 63, wv = wave_id();
  const int nr = d.nrhs;
  const long long nel = (long long)d.n * nr;
  const int j0 = i - d.k > 0 ? i - d.k : 0;
  const int nw = START ? 0 : i - j0;
  T* __restrict__ V = (T*)d.V;
  const T* __restrict__ src = START ? nullptr : V + (long long)(i - 1) * d.ldv;
  T* __restrict__ dst = V + (long long)i * d.ldv;

  UpdCoef<QC> cf;
  if constexpr (QC == 1) {
#pragma unroll
    for (int sl = 0; sl < NSLOT; ++sl)
      cf.c1[sl] = START ? (sl == 0 ? 1.0 : 0.0) : (sl == 0 || sl <= nw ? cfl[sl] : 0.0);
  } else {
    // (step_scalars has set every slot, zeros beyond the window; the start
    // pass stores b itself)
    if (START)
      for (int x = tid; x < nr * NSLOT; x += BLOCK) cfl[x] = (x % NSLOT) == 0 ? 1.0 : 0.0;
    cf.tab = cfl;
  }

  const int snr = d.s * nr;
  const bool reg_acc = SK == SK_SRHT && srht_reg_slots<QC>() > 0 && d.sk_reg;
  // SRHT with 8 or more rhs (several rhs per grid row): sums kept by rhs
  // pairs.  With exactly 8 rhs the sums of the sampled rows p < QROWS BLOCK
  // live in registers (thread tid owns rows tid + a BLOCK), the others in
  // LDS, and the LDS this frees holds a second tile buffer for the
  // transform.  The host sizes LDS the same way.
  const bool qmajor = SK == SK_SRHT && QC > 1 && !reg_acc && nr >= EPT;
  constexpr int QROWS = srht_qrows(KT) > 0 ? srht_qrows(KT) : 1;   // register array size
  const bool q8 = qmajor && nr == EPT && srht_qrows(KT) > 0;
  const int rreg = q8 ? QROWS * BLOCK : 0;
  const int sacc = d.s > rreg ? d.s - rreg : 0;                      // sampled rows summed in LDS
  double* X = lds;                                                   // SRHT tile (padded)
  double* X2 = q8 ? X + padx(TILE) : X;                              // second tile buffer
  double* acc = lds + (SK == SK_SRHT ? (q8 ? 2 : 1) * padx(TILE) : 0);   // sketch sums (LDS part)
  const int lslots = sacc * nr;   // = snr except on the 8-rhs path
  // sparse sign: one accumulator per wave when the host sized LDS for it, so
  // that the LDS atomics of different waves never meet (fixed order)
  const int nsl = (SK == SK_SPARSE && NW > 1 && d.sk_slices == NW) ? NW : 1;
  double* acc_w = acc + (nsl > 1 ? wv * snr : 0);
  int* rows_l = (int*)(acc + (reg_acc ? 0 : lslots * nsl));          // sampled SRHT rows
  if (!reg_acc)
    for (int x = tid; x < lslots * nsl; x += BLOCK) acc[x] = 0.0;
  if (SK == SK_SRHT)
    for (int x = tid; x < d.s; x += BLOCK) rows_l[x] = d.srht_rows[x];
  double racc[RA];
#pragma unroll
  for (int a = 0; a < RA; ++a) racc[a] = 0.0;
  double qacc[QROWS][EPT];   // register sums of the 8-rhs path: sampled rows tid + a BLOCK
#pragma unroll
  for (int a = 0; a < QROWS; ++a)
#pragma unroll
    for (int q = 0; q < EPT; ++q) qacc[a][q] = 0.0;
  __syncthreads();

  double nrm[QC];
#pragma unroll
  for (int c = 0; c < QC; ++c) nrm[c] = 0.0;
  const bool fast_ok = !START && OP == OP_STENCIL && nw == KT && stencil_fast_ok<T>(d);
  const long long reach = stencil_reach(d);
  const TileWalk tw = tile_walk(d, blk);
  auto interior = [&](int tt) {
    return fast_ok && ((long long)tt << LT) >= reach && (((long long)tt + 1) << LT) + reach <= nel;
  };
  // FP32 storage, one rhs: the source and window values of the block's next
  // interior tile are loaded before this tile's store and sketch (LDS) phase,
  // so that they are in flight meanwhile (the barriers of that phase wait for
  // LDS operations only).  With several rhs the extra registers would cost a
  // wave per SIMD (measured: slower).
  constexpr bool PF = sizeof(T) == 4 && QC == 1;
  T pc[EPT], pwin[KT > 1 ? KT - 1 : 1][EPT];
  int pf_t = -1;   // the tile whose values pc / pwin hold
  auto prefetch = [&](int tt) {
    const long long ee = ((long long)tt << LT) + (long long)tid * EPT;
    load8r(src + ee, pc);
#pragma unroll
    for (int jj = 0; jj < KT - 1; ++jj) load8r(V + (long long)(j0 + jj) * d.ldv + ee, pwin[jj]);
    pf_t = tt;
  };
  if (PF && tw.u0 < tw.uhi && interior(walk_tile(d, tw, tw.u0))) prefetch(walk_tile(d, tw, tw.u0));
  for (int iw = tw.u0; iw < tw.uhi; iw += tw.step) {
    const int t = walk_tile(d, tw, iw);
    const long long e = ((long long)t << LT) + (long long)tid * EPT;
    double uu[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) uu[j] = 0.0;
    if (e < nel) {
      double u[EPT];
      if (START) {
        get8(d.b, e, nel, u);
      } else if (interior(t)) {
        // interior tile, full window: all loads first, no branches; loaded
        // values stay in the storage type until used
        T c[EPT], win[KT > 1 ? KT - 1 : 1][EPT];
        double w[EPT];
        if (PF && pf_t == t) {
#pragma unroll
          for (int j = 0; j < EPT; ++j) c[j] = pc[j];
#pragma unroll
          for (int jj = 0; jj < KT - 1; ++jj)
#pragma unroll
            for (int j = 0; j < EPT; ++j) win[jj][j] = pwin[jj][j];
        } else {
          load8r(src + e, c);
#pragma unroll
          for (int jj = 0; jj < KT - 1; ++jj) load8r(V + (long long)(j0 + jj) * d.ldv + e, win[jj]);
        }
        stencil8_fast_raw(d, src, e, c, w);
        // same order of operations as the general path below
#pragma unroll
        for (int j = 0; j < EPT; ++j) u[j] = cf.get(tid, j, nr, 0) * w[j];
#pragma unroll
        for (int jj = 0; jj < KT - 1; ++jj)
#pragma unroll
          for (int j = 0; j < EPT; ++j) u[j] -= cf.get(tid, j, nr, 1 + jj) * (double)win[jj][j];
#pragma unroll
        for (int j = 0; j < EPT; ++j) u[j] -= cf.get(tid, j, nr, KT) * (double)c[j];
        if (PF) {
          pf_t = -1;
          const int iwn = iw + tw.step;
          if (iwn < tw.uhi) {
            const int tn = walk_tile(d, tw, iwn);
            if (interior(tn)) prefetch(tn);
          }
        }
      } else {
        double w[EPT];
        if (OP == OP_STENCIL) {
          double c[EPT];
          get8(src, e, nel, c);
          stencil8(d, src, e, nel, c, w);
        } else {
          get8(d.wbuf, e, nel, w);
        }
#pragma unroll
        for (int j = 0; j < EPT; ++j) u[j] = cf.get(tid, j, nr, 0) * w[j];
#pragma unroll
        for (int jj = 0; jj < KT; ++jj) {
          if (jj < nw) {
            double vj[EPT];
            get8(V + (long long)(j0 + jj) * d.ldv, e, nel, vj);
#pragma unroll
            for (int j = 0; j < EPT; ++j) u[j] -= cf.get(tid, j, nr, 1 + jj) * vj[j];
          }
        }
      }
      if (e + EPT <= nel) {
        store8(dst + e, u, uu);
      } else {
#pragma unroll
        for (int j = 0; j < EPT; ++j)
          if (e + j < nel) {
            const T ut = (T)u[j];
            dst[e + j] = ut;
            uu[j] = (double)ut;
          }
      }
#pragma unroll
      for (int j = 0; j < EPT; ++j) nrm[slot_of<QC>(j)] += uu[j] * uu[j];
      if (SK == SK_SPARSE) {
        // the column of Theta is a function of the row: hashed once per row
        // (the rhs of a row are consecutive elements)
        int rows[ZMAX];
        unsigned long long sb = 0;
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          if (e + j < nel) {
            const int r = (int)((e + j) >> d.lognrhs);
            const int q = (int)((e + j) & (nr - 1));
            if (j == 0 || q == 0) sparse_sign_column(d.key_a, d.key_b, r, d.s, d.zeta, rows, &sb);
#pragma unroll
            for (int tt = 0; tt < ZMAX; ++tt)
              if (tt < d.zeta) atomicAdd(&acc_w[rows[tt] * nr + q], ((sb >> tt) & 1ull) ? -uu[j] : uu[j]);
          }
        }
      }
    }
    if (SK == SK_SRHT) {
      // D signs (hashed once per row: the rhs of a row are consecutive
      // elements), then the transform of the tile along rows
      bool neg = false;
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const long long ej = e + j;
        if (j == 0 || (ej & (nr - 1)) == 0) neg = (sm64_out(d.key_a, (unsigned long long)(ej >> d.lognrhs)) >> 63) != 0;
        if (neg) uu[j] = -uu[j];
      }
      double* XF = X;   // the buffer holding the transformed tile
      if (q8) XF = fwht_tile2<LT>(uu, X, X2, d.lognrhs);
      else fwht_tile<LT>(uu, X, d.lognrhs);
      // sampled rows r = (r_hi, r_lo): contribution (-1)^popcount(r_hi & t) * X[r_lo]
      if (reg_acc) {
        const int lomask = d.rows_per_tile - 1;
#pragma unroll
        for (int a = 0; a < RA; ++a) {
          const int pq = tid + a * BLOCK;
          if (pq < snr) {
            const int rr = rows_l[pq >> d.lognrhs];
            const int par = __popc((unsigned)(rr >> d.log_rows) & (unsigned)t) & 1;
            const double v = X[padx(((rr & lomask) << d.lognrhs) + (pq & (nr - 1)))];
            racc[a] += par ? -v : v;
          }
        }
      } else {
        const int lomask = d.rows_per_tile - 1;
        if (qmajor) {
          // several rhs: thread tid owns the sampled rows p = tid + a BLOCK
          // with all their rhs; the rhs of a row are consecutive in the tile,
          // so one row index, one sign and one address serve nr sums.  The
          // LDS accumulators are kept by rhs pairs (sum (p, q) at
          // ((q/2) sacc + p - rreg) 2 + q mod 2), so each access moves two
          // sums and the lanes of a wave touch consecutive 16-byte words.
          // The sign is applied as a mask on the sign bit of the values.
#pragma unroll
          for (int a = 0; a < QROWS; ++a) {
            if (tid + a * BLOCK < rreg && tid + a * BLOCK < d.s) {
              const int rr = rows_l[tid + a * BLOCK];
              const int smask = (int)((unsigned)__popc((unsigned)(rr >> d.log_rows) & (unsigned)t) << 31);
              const double* xp = XF + padx((rr & lomask) << d.lognrhs);
#pragma unroll
              for (int q = 0; q < EPT; ++q)
                qacc[a][q] += __hiloint2double(__double2hiint(xp[q]) ^ smask, __double2loint(xp[q]));
            }
          }
          for (int p = rreg + tid; p < d.s; p += BLOCK) {
            const int rr = rows_l[p];
            const int smask = (int)((unsigned)__popc((unsigned)(rr >> d.log_rows) & (unsigned)t) << 31);
            const int b = (rr & lomask) << d.lognrhs;
            for (int q0 = 0; q0 < nr; q0 += EPT) {
              // 8 consecutive elements from a multiple of 8 share one
              // padding group of the tile
              const double* xp = XF + padx(b + q0);
              double2* ap = reinterpret_cast<double2*>(acc) + (q0 / 2) * sacc + (p - rreg);
              double xv[EPT];
              double2 av[EPT / 2];
#pragma unroll
              for (int q = 0; q < EPT; ++q) xv[q] = xp[q];
#pragma unroll
              for (int h = 0; h < EPT / 2; ++h) av[h] = ap[h * sacc];
#pragma unroll
              for (int h = 0; h < EPT / 2; ++h) {
                double2 o;
                o.x = av[h].x + __hiloint2double(__double2hiint(xv[2 * h]) ^ smask, __double2loint(xv[2 * h]));
                o.y = av[h].y + __hiloint2double(__double2hiint(xv[2 * h + 1]) ^ smask, __double2loint(xv[2 * h + 1]));
                ap[h * sacc] = o;
              }
            }
          }
        } else
        for (int pq0 = tid; pq0 < snr; pq0 += SK_BATCH * BLOCK) {
          double v[SK_BATCH], o[SK_BATCH];
#pragma unroll
          for (int u = 0; u < SK_BATCH; ++u) {
            const int pq = pq0 + u * BLOCK;
            v[u] = 0.0;
            o[u] = 0.0;
            if (pq < snr) {
              const int rr = rows_l[pq >> d.lognrhs];
              const int par = __popc((unsigned)(rr >> d.log_rows) & (unsigned)t) & 1;
              const double x = X[padx(((rr & lomask) << d.lognrhs) + (pq & (nr - 1)))];
              v[u] = par ? -x : x;
              o[u] = acc[pq];
            }
          }
#pragma unroll
          for (int u = 0; u < SK_BATCH; ++u) {
            const int pq = pq0 + u * BLOCK;
            if (pq < snr) acc[pq] = o[u] + v[u];
          }
        }
      }
      // the next tile's transform writes X first: after a read of X, a
      // barrier; after a read of X2 none is needed (the next write of X2
      // follows the next transform's first barrier)
      if (XF == X) __syncthreads();
    }
  }
  __syncthreads();
  double* skp = d.skpart + (long long)(i & 1) * d.skstride;
  if (reg_acc) {
#pragma unroll
    for (int a = 0; a < RA; ++a) {
      const int pq = tid + a * BLOCK;
      if (pq < snr) skp[((long long)(pq >> 3) * d.nblk + blk) * 8 + (pq & 7)] = racc[a];
    }
  } else if (qmajor) {
#pragma unroll
    for (int a = 0; a < QROWS; ++a)
      if (tid + a * BLOCK < rreg && tid + a * BLOCK < d.s) {
        const int p = tid + a * BLOCK;
#pragma unroll
        for (int q = 0; q < EPT; ++q) {
          const int pq = p * EPT + q;
          skp[((long long)(pq >> 3) * d.nblk + blk) * 8 + (pq & 7)] = qacc[a][q];
        }
      }
    for (int x = tid; x < lslots; x += BLOCK) {
      const int q = x & (nr - 1), pl = x >> d.lognrhs;
      const int pq = (pl + rreg) * nr + q;
      skp[((long long)(pq >> 3) * d.nblk + blk) * 8 + (pq & 7)] = acc[(((q >> 1) * sacc + pl) << 1) + (q & 1)];
    }
  } else {
    for (int pq = tid; pq < snr; pq += BLOCK) {
      double a = acc[pq];
      for (int sl = 1; sl < nsl; ++sl) a += acc[sl * snr + pq];
      skp[((long long)(pq >> 3) * d.nblk + blk) * 8 + (pq & 7)] = a;
    }
  }

  // norm partials per rhs
  for (int q = 0; q < nr; ++q) {
    double a = 0.0;
#pragma unroll
    for (int c = 0; c < QC; ++c)
      if (rhs_of<QC>(tid, c, nr) == q) a += nrm[c];
    a = wave_sum_all(a);
    if (lane == 0) nred[wv][q] = a;
  }
  __syncthreads();
  double* npw = d.npart + (long long)(i & 1) * d.nblk * nr;
  for (int q = tid; q < nr; q += BLOCK) {
    double t = 0.0;
    for (int w = 0; w < NW; ++w) t += nred[w][q];
    npw[(long long)q * d.nblk + blk] = t;   // column-major, as the dot partials
  }
}

// ------------------------------------------------------------------ combine
// out = sum_j cf_j u_j with cf_j = beta c_j / eta_j (FP64 accumulation).
// Full chunks issue four basis-vector loads at a time; with one right-hand
// side (NR1) the weights are uniform values.
template <typename T, bool NR1>
__global__ void __launch_bounds__(256) k_combine(SolveDev d, const double* __restrict__ cf, int mmax,
                                                 double* __restrict__ out) {
  const T* __restrict__ V = (const T*)d.V;
  const long long nel = (long long)d.n * d.nrhs;
  const int nr = d.nrhs;
  const long long cld = d.m + 1;
  for (long long e = ((long long)blockIdx.x * 256 + threadIdx.x) * EPT; e < nel;
       e += (long long)gridDim.x * 256 * EPT) {
    long long cb[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) cb[j] = NR1 ? 0 : (long long)((e + j) & (nr - 1)) * cld;
    double a[EPT];
#pragma unroll
    for (int j = 0; j < EPT; ++j) a[j] = 0.0;
    int jv = 0;
    if (e + EPT <= nel) {
      for (; jv + 4 <= mmax; jv += 4) {
        double v[4][EPT];
#pragma unroll
        for (int u = 0; u < 4; ++u) load8(V + (long long)(jv + u) * d.ldv + e, v[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int j = 0; j < EPT; ++j) a[j] += cf[cb[j] + jv + u] * v[u][j];
      }
    }
    for (; jv < mmax; ++jv) {
      double v[EPT];
      get8(V + (long long)jv * d.ldv, e, nel, v);
#pragma unroll
      for (int j = 0; j < EPT; ++j) a[j] += cf[cb[j] + jv] * v[j];
    }
    if (e + EPT <= nel) {
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        double2 o;
        o.x = a[2 * h];
        o.y = a[2 * h + 1];
        *reinterpret_cast<double2*>(out + e + 2 * h) = o;
      }
    } else {
      for (int j = 0; j < EPT; ++j)
        if (e + j < nel) out[e + j] = a[j];
    }
  }
}

}  // namespace fab
