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
// One workgroup per right-hand side and variant (256 threads).  Up to m = 128
// H_hat is held in registers (a 4-wave column split) and each term costs one
// pass with one barrier; above, H_hat is read from the per-rhs workspace in
// global memory, threads (r, h) for rows r and column halves h, two barriers
// per term.
#include "fab_dev.h"

namespace fab {

namespace {

constexpr int EMAXM = 512;
constexpr double RHO_MAX = 4.0;    // scaled norm per step
constexpr double TAYLOR_TOL = 1e-18;
constexpr int KMAX_TAYLOR = 64;
// Work bound: at most EXP_MAX_STEPS scaling steps (||alpha H_hat||_1 <=
// RHO_MAX * EXP_MAX_STEPS = 16384); beyond it the kernel stores NaN and
// reports INFO_FAIL = 3 (the solve then returns FAB_ENUMERIC) instead of
// running for a time proportional to the norm (a least-squares correction
// of an ill-conditioned basis can make ||H_hat|| arbitrarily large).
constexpr double EXP_MAX_STEPS = 4096.0;

// S, K and ||B||_1 for B = alpha H_hat (H_hat m x m, column-major); every
// thread of the 256-thread workgroup gets the same values.
__device__ __forceinline__ void taylor_plan(int m, const double* H, double alpha, double* red, int* Sout, int* Kout,
                                            double* nrm_out) {
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
  *nrm_out = nrm;
  const double Sd = ceil(nrm / RHO_MAX);
  if (!(Sd <= EXP_MAX_STEPS)) {   // also NaN
    *Sout = 0;
    *Kout = 0;
    return;
  }
  int S = (int)Sd;
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
  *Sout = S;
  *Kout = K;
}

// The result when the norm is beyond the work bound: NaN, INFO_FAIL = 3.
__device__ void taylor_refuse(int m, double nrm, double* out, double* info) {
  for (int r = threadIdx.x; r < m; r += 256) out[r] = __builtin_nan("");
  if (threadIdx.x == 0) {
    info[INFO_FAIL] = 3.0;
    info[INFO_NSQ] = 0.0;
    info[INFO_SCHUR_IT] = 0.0;
    info[INFO_NRM] = nrm;
  }
}

// m <= 128: H_hat in registers.  Wave w owns columns [w cw, (w+1) cw) with
// cw = ceil(m/4) <= 32, lane l owns rows l and l + 64 of those columns, and
// lane l < cw owns entry w cw + l of the vectors x and t.  A term
// t_k = (B/S) t_{k-1} / k is one pass: every lane forms the partial sums of
// its two rows over its wave's columns (the t entries broadcast from their
// owner lanes), writes them to LDS, one barrier, and each owner lane adds the
// four waves' partials of its entry (double-buffered partials, so the next
// term's writes never meet a slower wave's reads).
__device__ void taylor_action_regs(int m, const double* __restrict__ H, double alpha, double* part /*[2][4][128]*/,
                                   double* out, double* info, double* red) {
  const int tid = threadIdx.x, lane = tid & 63, w = wave_id();
  int S, K;
  double nrm;
  taylor_plan(m, H, alpha, red, &S, &K, &nrm);
  if (S == 0) {
    taylor_refuse(m, nrm, out, info);
    return;
  }
  const double bscale = alpha / S;
  const int cw = (m + 3) / 4, cb = w * cw;
  double h0[32], h1[32];
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const int c = cb + j;
    const bool okc = j < cw && c < m;
    h0[j] = (okc && lane < m) ? H[lane + (long long)c * m] : 0.0;
    h1[j] = (okc && lane + 64 < m) ? H[lane + 64 + (long long)c * m] : 0.0;
  }
  const int myc = cb + lane;
  const bool own = lane < cw && myc < m;
  double x = (own && myc == 0) ? 1.0 : 0.0;   // x_0 = e_1
  int buf = 0;
  for (int step = 0; step < S; ++step) {
    double t = x;
    for (int k = 1; k <= K; ++k) {
      double p0 = 0.0, p1 = 0.0, q0 = 0.0, q1 = 0.0;
#pragma unroll
      for (int j = 0; j < 32; j += 2) {
        const double ta = readlane_d(t, j), tb = readlane_d(t, j + 1);
        p0 += h0[j] * ta;
        p1 += h1[j] * ta;
        q0 += h0[j + 1] * tb;
        q1 += h1[j + 1] * tb;
      }
      double* pb = part + buf * 512 + w * 128;
      pb[lane] = p0 + q0;
      pb[lane + 64] = p1 + q1;
      __syncthreads();
      const double* pr = part + buf * 512;
      const double v = own ? (((pr[myc] + pr[128 + myc]) + pr[256 + myc]) + pr[384 + myc]) * (bscale / k) : 0.0;
      t = v;
      x += v;
      buf ^= 1;
    }
  }
  if (own) out[myc] = x;
  if (tid == 0) {
    info[INFO_NSQ] = S;        // scaling steps
    info[INFO_SCHUR_IT] = K;   // Taylor degree
    info[INFO_NRM] = nrm;      // ||alpha H_hat||_1
  }
}

// m > 128: H_hat read from global memory, rows split between two column
// halves per thread.
template <typename Ptr>
__device__ __forceinline__ void taylor_action(int m, Ptr H, double alpha, double* xs, double* ts, double* part,
                                              double* out, double* info, double* red) {
  const int tid = threadIdx.x;
  int S, K;
  double nrm;
  taylor_plan(m, H, alpha, red, &S, &K, &nrm);
  if (S == 0) {
    taylor_refuse(m, nrm, out, info);
    return;
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
        // four independent chains, loads of two groups in flight: the term
        // is bound by LDS latency, not by arithmetic
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int c = c0;
#pragma unroll 2
        for (; c + 3 < c1; c += 4) {
          const double h0 = H[r + (long long)c * m], h1 = H[r + (long long)(c + 1) * m];
          const double h2 = H[r + (long long)(c + 2) * m], h3 = H[r + (long long)(c + 3) * m];
          const double t0 = ts[c], t1 = ts[c + 1], t2 = ts[c + 2], t3 = ts[c + 3];
          a0 += h0 * t0;
          a1 += h1 * t1;
          a2 += h2 * t2;
          a3 += h3 * t3;
        }
        for (; c < c1; ++c) a0 += H[r + (long long)c * m] * ts[c];
        part[h * EMAXM + r] = (a0 + a1) + (a2 + a3);
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
  const int q = blockIdx.x, v = blockIdx.y;
  const DenseVariant dv = dense_variant(d, g, q, v);
  const int m = dv.dim;
  if (m == 0) return;
  const double* Hh = dv.H;
  double* c = dv.c;
  double* info = v == 0 ? dv.info : dv.scratch;   // the variants' scalars are not reported
  __shared__ double xs[EMAXM], ts[EMAXM], part[2 * EMAXM];
  __shared__ double red[4];
  if (m <= 128) taylor_action_regs(m, Hh, g.alpha, part, c, info, red);
  else taylor_action(m, Hh, g.alpha, xs, ts, part, c, info, red);
}

size_t exp_lds_bytes(int m) {
  (void)m;
  return 0;
}

hipError_t exp_launch(const SolveDev& d, const DenseDev& g, hipStream_t st) {
  hipLaunchKernelGGL(k_exp_taylor, dim3(d.nrhs, g.nvar), dim3(256), exp_lds_bytes(d.m), st, d, g);
  return hipGetLastError();
}

hipError_t exp_set_attributes() { return hipSuccess; }

}  // namespace fab
