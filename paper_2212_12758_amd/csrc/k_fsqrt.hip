// (H_hat + sigma I)^{+-1/2} e_1 by quadrature of a resolvent integral.
//
// With B = H_hat + sigma I (spectrum off the closed negative real axis),
//     B^{-1/2} = (2/pi) int_0^inf (t^2 I + B)^{-1} dt,
//     B^{+1/2} = (2/pi) int_0^inf B (t^2 I + B)^{-1} dt,
// and t = e^u turns both into integrals over the real line whose integrands
// decay exponentially at both ends and are analytic in a strip around the
// real axis, so the trapezoidal rule with step h converges exponentially
// (Trefethen & Weideman, SIAM Rev. 56 (2014) 385-458).  Nodes u_j = u_lo + j h:
//     f(B) e_1 ~ (2 h / pi) sum_j e^{u_j} [B] x_j,   x_j = (e^{2 u_j} I + B)^{-1} e_1.
// h = 1/8 makes the discretisation error below 1e-16 for spectra in the
// closed right half-plane; u_lo, u_hi bound the truncated tails by 1e-16
// relative to the result (u_hi from ||B||_1, u_lo from ||B^{-1} e_1|| for
// the inverse square root).
//
// H_hat is upper Hessenberg (Hessenberg H_m plus a change of its last column,
// eq. (6)), so each shifted solve is O(m^2): rotations of adjacent columns
// from the right, zeroing the subdiagonal bottom-up, give (e^{2u} I + B) G = T
// upper triangular, hence x = G T^{-1} e_1 = G e_1 / T_00; G e_1 is a running
// product of the rotations' sines and cosines.  One wave per node, the
// current column held in registers (rows over lanes), no matrix storage.
//
//   k_fs_setup  per (rhs, variant): ||B||_1, B^{-1} e_1, the node range.
//   k_fs_nodes  per (rhs, variant, block): its nodes, summed per block.
//   k_fs_sum    per (rhs, variant): the block sums in a fixed order.
#include "fab_dev.h"

namespace fab {

namespace {

constexpr int FS_MAXR = 8;        // rows per lane: order <= 512
constexpr int FS_LDS_M = 128;     // H staged in LDS up to this order
constexpr int FS_BLOCKS = 64;     // node blocks per (rhs, variant)
constexpr int FS_WAVES = 4;       // waves (nodes at a time) per block
constexpr int FS_MAXN = 2048;     // node cap
constexpr double FS_H = 0.125;
constexpr double FS_TAIL = 36.8;  // -log(1e-16)

struct FsParams {
  double u_lo, h;
  int n;
};

__device__ inline double wsum64(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// x = (B + tau I)^{-1} e_1 for the upper Hessenberg B = H + sigma I (order m,
// ld m), rows r = lane + 64 u in x[u].  Returns false when T_00 = 0.
template <int RR>
__device__ bool hess_shifted_solve(int m, const double* __restrict__ H, double shift, double* x) {
  constexpr int FS_MAXR = RR;   // rows per lane in this instantiation
  const int lane = threadIdx.x & 63;
  double cur[FS_MAXR], cs[FS_MAXR], sn[FS_MAXR];
#pragma unroll
  for (int u = 0; u < FS_MAXR; ++u) {
    const int r = lane + 64 * u;
    cur[u] = r < m ? H[r + (long long)(m - 1) * m] + (r == m - 1 ? shift : 0.0) : 0.0;
    cs[u] = 1.0;
    sn[u] = 0.0;
  }
  // column k-1 (rows 0..k) is loaded one step ahead
  double nxt[FS_MAXR];
#pragma unroll
  for (int u = 0; u < FS_MAXR; ++u) {
    const int r = lane + 64 * u;
    nxt[u] = (m >= 2 && r <= m - 1) ? H[r + (long long)(m - 2) * m] + (r == m - 2 ? shift : 0.0) : 0.0;
  }
  for (int k = m - 1; k >= 1; --k) {
    double col[FS_MAXR];
#pragma unroll
    for (int u = 0; u < FS_MAXR; ++u) col[u] = nxt[u];
    if (k >= 2) {
#pragma unroll
      for (int u = 0; u < FS_MAXR; ++u) {
        const int r = lane + 64 * u;
        nxt[u] = r <= k - 1 ? H[r + (long long)(k - 2) * m] + (r == k - 2 ? shift : 0.0) : 0.0;
      }
    }
    const int ku = k >> 6, kl = k & 63;
    double a_src = col[0], b_src = cur[0];
#pragma unroll
    for (int u = 1; u < FS_MAXR; ++u)
      if (ku == u) { a_src = col[u]; b_src = cur[u]; }
    const double a = readlane_d(a_src, kl), bb = readlane_d(b_src, kl);
    const double rr = sqrt(a * a + bb * bb);
    const double inv = rr > 0.0 ? 1.0 / rr : 0.0;
    const double c = rr > 0.0 ? bb * inv : 1.0, s = rr > 0.0 ? a * inv : 0.0;
#pragma unroll
    for (int u = 0; u < FS_MAXR; ++u) {
      const int r = lane + 64 * u;
      cur[u] = r < k ? c * col[u] - s * cur[u] : 0.0;
      if (r == k) { cs[u] = c; sn[u] = s; }
    }
  }
  const double t00 = readlane_d(cur[0], 0);
  // G e_1: v_0 = c_1, v_j = c_{j+1} prod_{l<=j} (-s_l), v_{m-1} = prod_{l<m} (-s_l);
  // prefix products over the rows held by lanes, then across lanes in order
  double pre[FS_MAXR];
  double carry = 1.0;
#pragma unroll
  for (int u = 0; u < FS_MAXR; ++u) {
    // inclusive prefix product of (-s_r) over r = 64u .. 64u + lane (r >= 1)
    const int r = lane + 64 * u;
    double p = (r >= 1 && r < m) ? -sn[u] : 1.0;
    for (int off = 1; off < 64; off <<= 1) {
      const double o = __shfl_up(p, off, 64);
      if (lane >= off) p *= o;
    }
    pre[u] = p * carry;
    carry *= __shfl(p, 63, 64);
  }
  bool ok = t00 != 0.0 && isfinite(t00);
#pragma unroll
  for (int u = 0; u < FS_MAXR; ++u) {
    const int r = lane + 64 * u;
    // c_{r+1} lives in the lane holding row r + 1 (every lane shuffles)
    const double cn_lo = __shfl_down(cs[u], 1, 64);
    const double cn_hi = __shfl(cs[u + 1 < FS_MAXR ? u + 1 : u], 0, 64);
    const double cn = lane < 63 ? cn_lo : (u + 1 < FS_MAXR ? cn_hi : 1.0);
    const double v = r == m - 1 ? pre[u] : cn * pre[u];
    x[u] = r < m ? (ok ? v / t00 : 0.0) : 0.0;
  }
  return ok;
}

__device__ inline double* fs_partials(double* fq, int m, int q, int v) {
  return fq + ((long long)q * 3 + v) * FS_BLOCKS * (m + 1);
}

// Copy the m x m matrix to LDS with eight loads in flight per thread.
__device__ inline void fs_stage(const double* __restrict__ H, double* Hl, int m, int nthreads) {
  const long long n2 = (long long)m * m;
  long long x = threadIdx.x;
  for (; x + 7LL * nthreads < n2; x += 8LL * nthreads) {
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = H[x + u * nthreads];
#pragma unroll
    for (int u = 0; u < 8; ++u) Hl[x + u * nthreads] = t[u];
  }
  for (; x < n2; x += nthreads) Hl[x] = H[x];
}

template <int RR, bool STAGED>
__global__ void __launch_bounds__(64) k_fs_setup(SolveDev d, DenseDev g, double* fq) {
  constexpr int FS_MAXR = RR;
  extern __shared__ double hl[];
  const int q = blockIdx.x, v = blockIdx.y, lane = threadIdx.x;
  const DenseVariant dv = dense_variant(d, g, q, v);
  const int m = dv.dim;
  FsParams* P = (FsParams*)dv.scratch;
  if (m == 0) {
    if (lane == 0) P->n = 0;
    return;
  }
  if (STAGED) {
    fs_stage(dv.H, hl, m, 64);
    __syncthreads();
  }
  const double* H = STAGED ? (const double*)hl : dv.H;
  // ||B||_1
  double cmax = 0.0;
  for (int c = lane; c < m; c += 64) {
    double a = 0.0;
    for (int r = 0; r < m; ++r) a += fabs(H[r + (long long)c * m] + (r == c ? g.sigma : 0.0));
    cmax = fmax(cmax, a);
  }
  for (int off = 32; off >= 1; off >>= 1) cmax = fmax(cmax, __shfl_xor(cmax, off, 64));
  const double nb = fmax(cmax, 1e-300);
  double u_lo;
  if (g.p < 0.0) {
    double x[FS_MAXR];
    const bool ok = hess_shifted_solve<RR>(m, H, g.sigma, x);
    double n2 = 0.0;
#pragma unroll
    for (int u = 0; u < FS_MAXR; ++u) n2 += x[u] * x[u];
    n2 = wsum64(n2);
    const double xn = ok ? sqrt(n2) : 1e300;
    u_lo = -FS_TAIL - log(fmax(xn * sqrt(nb), 1e-300));
  } else {
    u_lo = 0.5 * log(nb) - FS_TAIL - 10.0;
  }
  const double u_hi = 0.5 * log(nb) + FS_TAIL;
  double h = FS_H;
  int n = (int)ceil((u_hi - u_lo) / h) + 1;
  if (!(n > 0)) n = 1;
  if (n > FS_MAXN) {
    n = FS_MAXN;
    h = (u_hi - u_lo) / (n - 1);
  }
  if (lane == 0) {
    P->u_lo = u_lo;
    P->h = h;
    P->n = isfinite(u_lo) && isfinite(u_hi) ? n : -1;
  }
}

template <int RR, bool STAGED>
__global__ void __launch_bounds__(64 * FS_WAVES) k_fs_nodes(SolveDev d, DenseDev g, double* fq) {
  constexpr int FS_MAXR = RR;
  extern __shared__ double hl[];
  const int q = blockIdx.x, v = blockIdx.y, blk = blockIdx.z;
  const int lane = threadIdx.x & 63, wv = wave_id();
  const DenseVariant dv = dense_variant(d, g, q, v);
  const int m = dv.dim;
  const FsParams P = *(const FsParams*)dv.scratch;
  __shared__ double red[FS_WAVES][FS_MAXR * 64];
  if (STAGED && m > 0 && P.n > blk * FS_WAVES) {
    fs_stage(dv.H, hl, m, 64 * FS_WAVES);
    __syncthreads();
  }
  const double* H = STAGED ? (const double*)hl : dv.H;
  double acc[FS_MAXR];
#pragma unroll
  for (int u = 0; u < FS_MAXR; ++u) acc[u] = 0.0;
  if (m > 0 && P.n > 0) {
    for (int j = blk * FS_WAVES + wv; j < P.n; j += FS_BLOCKS * FS_WAVES) {
      const double uj = P.u_lo + j * P.h;
      const double et = exp(uj);
      double x[FS_MAXR];
      hess_shifted_solve<RR>(m, H, g.sigma + et * et, x);
      if (g.p > 0.0) {
        // B x: rows over lanes, x_c read from the lane that holds it
        double y[FS_MAXR];
#pragma unroll
        for (int u = 0; u < FS_MAXR; ++u) y[u] = 0.0;
        for (int c = 0; c < m; ++c) {
          const int cu = c >> 6;
          double src = x[0];
#pragma unroll
          for (int u = 1; u < FS_MAXR; ++u)
            if (cu == u) src = x[u];
          const double xc = readlane_d(src, c & 63);
#pragma unroll
          for (int u = 0; u < FS_MAXR; ++u) {
            const int r = lane + 64 * u;
            if (r < m && r <= c + 1) y[u] += (H[r + (long long)c * m] + (r == c ? g.sigma : 0.0)) * xc;
          }
        }
#pragma unroll
        for (int u = 0; u < FS_MAXR; ++u) x[u] = y[u];
      }
#pragma unroll
      for (int u = 0; u < FS_MAXR; ++u) acc[u] += et * x[u];
    }
  }
#pragma unroll
  for (int u = 0; u < FS_MAXR; ++u) red[wv][lane + 64 * u] = acc[u];
  __syncthreads();
  double* out = fs_partials(fq, d.m, q, v) + (long long)blk * (d.m + 1);
  for (int r = threadIdx.x; r < m; r += 64 * FS_WAVES) {
    double t = 0.0;
    for (int w = 0; w < FS_WAVES; ++w) t += red[w][r];
    out[r] = t;
  }
}

__global__ void __launch_bounds__(256) k_fs_sum(SolveDev d, DenseDev g, double* fq) {
  const int q = blockIdx.x, v = blockIdx.y;
  const DenseVariant dv = dense_variant(d, g, q, v);
  const int m = dv.dim;
  if (m == 0) return;
  const FsParams P = *(const FsParams*)dv.scratch;
  const double* part = fs_partials(fq, d.m, q, v);
  const double w = 2.0 * P.h / 3.14159265358979323846;
  __shared__ int nonfinite;
  if (threadIdx.x == 0) nonfinite = 0;
  __syncthreads();
  for (int r = threadIdx.x; r < m; r += 256) {
    double t = 0.0;
    for (int b = 0; b < FS_BLOCKS; ++b) t += part[(long long)b * (d.m + 1) + r];
    const double val = w * t;
    dv.c[r] = val;
    if (!isfinite(val)) nonfinite = 1;
  }
  __syncthreads();
  const bool bad = P.n <= 0 || nonfinite;
  if (bad)
    for (int r = threadIdx.x; r < m; r += 256) dv.c[r] = 0.0;
  if (threadIdx.x == 0) {
    if (bad) dv.info[v == 0 ? INFO_FAIL : INFO_VFAIL + v] = 2.0;
    if (v == 0) {
      dv.info[INFO_NSQ] = P.n;   // quadrature nodes
      dv.info[INFO_SCHUR_IT] = 0.0;
    }
  }
}

}  // namespace

size_t fsqrt_partials_doubles(int m, int nrhs) { return (size_t)nrhs * 3 * FS_BLOCKS * (m + 1); }

namespace {
// The planned order d.m bounds every variant's order: it picks the rows per
// lane and whether H fits in LDS.
template <int RR, bool STAGED>
void fs_launch_t(const SolveDev& d, const DenseDev& g, double* fq, hipStream_t st) {
  const size_t lds = STAGED ? (size_t)d.m * d.m * 8 : 0;
  hipLaunchKernelGGL((k_fs_setup<RR, STAGED>), dim3(d.nrhs, g.nvar), dim3(64), lds, st, d, g, fq);
  hipLaunchKernelGGL((k_fs_nodes<RR, STAGED>), dim3(d.nrhs, g.nvar, FS_BLOCKS), dim3(64 * FS_WAVES), lds, st, d, g,
                     fq);
}
}  // namespace

hipError_t fsqrt_launch(const SolveDev& d, const DenseDev& g, double* fq, hipStream_t st) {
  if (d.m > 64 * FS_MAXR) return hipErrorInvalidValue;
  if (d.m <= 64) fs_launch_t<1, true>(d, g, fq, st);
  else if (d.m <= FS_LDS_M) fs_launch_t<2, true>(d, g, fq, st);
  else if (d.m <= 256) fs_launch_t<4, false>(d, g, fq, st);
  else fs_launch_t<8, false>(d, g, fq, st);
  hipLaunchKernelGGL(k_fs_sum, dim3(d.nrhs, g.nvar), dim3(256), 0, st, d, g, fq);
  return hipGetLastError();
}

hipError_t fsqrt_set_attributes() {
  hipError_t e = hipSuccess, r;
  const int lds = FS_LDS_M * FS_LDS_M * 8;
  const void* ks[4] = {(const void*)k_fs_setup<1, true>, (const void*)k_fs_setup<2, true>,
                       (const void*)k_fs_nodes<1, true>, (const void*)k_fs_nodes<2, true>};
  for (const void* k : ks)
    if ((r = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, lds)) != hipSuccess) e = r;
  return e;
}

}  // namespace fab
