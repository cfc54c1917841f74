// exp(alpha H_hat) e_1, the matrix exponential the paper applies to the
// compressed matrix (Section 5 experiments), computed as the action of the
// exponential on a vector (Al-Mohy & Higham, SIAM J. Sci. Comput. 33 (2011)
// 488-511): with B = alpha H_hat, S = max(1, ceil(||B||_1 / RHO_MAX)) and
// rho = ||B||_1 / S,
//     x_0 = e_1,   x_{i+1} = T_K(B / S) x_i,   exp(B) e_1 = x_S,
// where T_K is the Taylor polynomial of degree K, the smallest degree whose
// first omitted term is bounded by rho^{K+1}/(K+1)! <= TAYLOR_TOL (the terms
// satisfy ||(B/S)^k x / k!||_1 <= rho^k/k! ||x||_1).  Only products of the
// small matrix with a vector are needed: no factorisation, no matrix products.
//
// One workgroup per right-hand side (256 threads).  H_hat is kept in LDS when
// the planned order fits (m <= 112), else read from the per-rhs workspace in
// global memory.  Each term costs one product: threads (r, h) for rows r and
// column halves h, two barriers.
#include "fab_dev.h"

namespace fab {

namespace {

constexpr int LDSM = 112;          // H_hat kept in LDS up to this order
constexpr int EMAXM = 512;
constexpr double RHO_MAX = 4.0;    // scaled norm per step
constexpr double TAYLOR_TOL = 1e-18;
constexpr int KMAX_TAYLOR = 64;

template <typename Ptr>
__device__ __forceinline__ void taylor_action(int m, Ptr H, double alpha, double* xs, double* ts, double* part,
                                              double* out, double* info, double* red) {
  const int tid = threadIdx.x;
  // ||B||_1 = |alpha| max_c sum_r |H_hat[r, c]|
  double cmax = 0.0;
  for (int c = tid; c < m; c += 256) {
    double a = 0.0;
    for (int r = 0; r < m; ++r) a += fabs(H[r + (long long)c * m]);
    cmax = fmax(cmax, a);
  }
  for (int off = 32; off >= 1; off >>= 1) cmax = fmax(cmax, __shfl_xor(cmax, off, 64));
  if ((tid & 63) == 0) red[tid >> 6] = cmax;
  __syncthreads();
  const double nrm = fmax(fmax(red[0], red[1]), fmax(red[2], red[3])) * fabs(alpha);
  int S = (int)ceil(nrm / RHO_MAX);
  if (S < 1) S = 1;
  const double rho = nrm / S;
  // degree: first omitted term rho^(K+1)/(K+1)! below the tolerance
  int K = 1;
  {
    double t = rho;   // rho^K / K!
    while (K < KMAX_TAYLOR) {
      const double nxt = t * rho / (K + 1);
      if (nxt <= TAYLOR_TOL) break;
      t = nxt;
      ++K;
    }
  }
  const double bscale = alpha / S;
  // thread (r, h): rows r = (tid & 127) + 128 j, column half h = tid >> 7
  const int h = tid >> 7, r0 = tid & 127;
  const int half = (m + 1) / 2, c0 = h * half, c1 = h ? m : half;
  for (int r = tid; r < m; r += 256) xs[r] = r == 0 ? 1.0 : 0.0;
  __syncthreads();
  for (int step = 0; step < S; ++step) {
    // x += sum_k t_k with t_0 = x, t_k = (B / S) t_{k-1} / k
    for (int r = tid; r < m; r += 256) ts[r] = xs[r];
    __syncthreads();
    for (int k = 1; k <= K; ++k) {
      const double f = bscale / k;
      for (int r = r0; r < m; r += 128) {
        double a0 = 0.0, a1 = 0.0;
        int c = c0;
        for (; c + 1 < c1; c += 2) {
          a0 += H[r + (long long)c * m] * ts[c];
          a1 += H[r + (long long)(c + 1) * m] * ts[c + 1];
        }
        if (c < c1) a0 += H[r + (long long)c * m] * ts[c];
        part[h * EMAXM + r] = a0 + a1;
      }
      __syncthreads();
      for (int r = tid; r < m; r += 256) {
        const double v = (part[r] + part[EMAXM + r]) * f;
        ts[r] = v;
        xs[r] += v;
      }
      __syncthreads();
    }
  }
  for (int r = tid; r < m; r += 256) out[r] = xs[r];
  if (tid == 0) {
    info[INFO_NSQ] = S;        // scaling steps
    info[INFO_SCHUR_IT] = K;   // Taylor degree
    info[INFO_NRM] = nrm;      // ||alpha H_hat||_1
  }
}

}  // namespace

__global__ void __launch_bounds__(256) k_exp_taylor(SolveDev d, DenseDev g) {
  const int q = blockIdx.x, tid = threadIdx.x, v = blockIdx.y;
  const DenseVariant dv = dense_variant(d, g, q, v);
  const int m = dv.dim;
  if (m == 0) return;
  const long long mm = (long long)m * m;
  const double* Hh = dv.H;
  double* c = dv.c;
  double* info = v == 0 ? dv.info : dv.scratch;   // the variants' scalars are not reported
  extern __shared__ double h_lds[];
  __shared__ double xs[EMAXM], ts[EMAXM], part[2 * EMAXM];
  __shared__ double red[4];
  // the dynamic LDS is sized for the planned order d.m (m_used <= d.m)
  if (d.m <= LDSM) {
    for (long long x = tid; x < mm; x += 256) h_lds[x] = Hh[x];
    __syncthreads();
    taylor_action(m, h_lds, g.alpha, xs, ts, part, c, info, red);
  } else {
    taylor_action(m, Hh, g.alpha, xs, ts, part, c, info, red);
  }
}

size_t exp_lds_bytes(int m) { return m <= LDSM ? (size_t)m * m * 8 : 0; }

hipError_t exp_launch(const SolveDev& d, const DenseDev& g, hipStream_t st) {
  hipLaunchKernelGGL(k_exp_taylor, dim3(d.nrhs, g.nvar), dim3(256), exp_lds_bytes(d.m), st, d, g);
  return hipGetLastError();
}

hipError_t exp_set_attributes() {
  return hipFuncSetAttribute((const void*)k_exp_taylor, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)((size_t)LDSM * LDSM * 8));
}

}  // namespace fab
