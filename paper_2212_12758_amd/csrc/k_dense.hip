// Small dense FP64 stages of the method, one workgroup per right-hand side:
//
//  k_gram   G = W^T W of the normalised sketch W = Theta V_{m+1} (many
//           workgroups).
//  k_lsq    the triangular factor R of W: Cholesky of G (whose last column
//           of R is [z; rho] with z = Q^T Theta v_{m+1}), in LDS when
//           s <= 448 and m + 1 <= 104, else in global memory; when a pivot
//           fails or R's diagonal spreads by more than 1e3, Householder QR of
//           W (in registers, or in global memory); y = R_m^{-1} z
//           (sketch-and-solve of the least-squares problem eq. (7), Remark 3)
//           by back substitution; the compression H_hat = H_m + h_{m+1,m} y
//           e_m^T (eq. (6)).
//  (exp(alpha H_hat) e_1 lives in k_expm.hip: the action of the exponential on
//   e_1 by a scaled truncated Taylor series.)
//  ((H_hat + sigma I)^{+-1/2} e_1 lives in k_fsqrt.hip: resolvent quadrature.)
//  k_fpoly  sum_j coef_j H_hat^j e_1 (polynomial test functions).
//  k_coef   combination weights beta c_j / eta_j for the final V c.
//
// All matrices are column-major with leading dimension m (or s) in a per-rhs
// workspace in global memory.
#include "fab_dev.h"

namespace fab {

hipError_t exp_launch(const SolveDev& d, const DenseDev& g, hipStream_t st);
hipError_t exp_set_attributes();

constexpr int DBLOCK = 256;
constexpr int MAXM = 512;

// Orders this wave's memory operations (LDS and global) without a workgroup
// barrier; used inside sections that only one wave executes.
__device__ inline void wave_order() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

__device__ inline double wsum(double v) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// block-wide sum; `sh` holds >= 4 doubles; every thread gets the result
__device__ inline double bsum(double v, double* sh) {
  const int lane = threadIdx.x & 63, wv = wave_id();
  v = wsum(v);
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double t = 0.0;
  const int nwv = (blockDim.x + 63) >> 6;
  for (int w = 0; w < nwv; ++w) t += sh[w];
  __syncthreads();
  return t;
}

__device__ inline int* st_mused(const SolveDev& d, int q) { return d.status + 4 + 2 * q; }
__device__ inline int* st_brk(const SolveDev& d, int q) { return d.status + 5 + 2 * q; }

// ----------------------------------------------------------------- sketched QR and least squares
constexpr int LBLOCK = 512;          // 8 waves
constexpr int LRS = 7;               // row slots per lane: rows lane + 64*rs  (s <= 448)
constexpr int LCS = 13;              // column slots per wave: cols wave + 8*cs (m + 1 <= 104)

// Householder QR of W (s x ncol, column-major, normalised sketch columns) held
// in registers; on exit R (ncol-1 x ncol-1 upper, ld mu) and z = first mu
// entries of the transformed last column are written to Rl / zl (LDS), and
// |r_jj| extremes to rmm.
__device__ void qr_registers(const double* __restrict__ S, const double* __restrict__ eta, int s, int ncol,
                             double* vsh, double* Rl, double* zl, double* tau_sh, double* rmm) {
  const int tid = threadIdx.x, lane = tid & 63, wv = wave_id();
  const int mu = ncol - 1;
  double a[LCS][LRS];
#pragma unroll
  for (int cs = 0; cs < LCS; ++cs) {
    const int c = wv + 8 * cs;
    const double e = c < ncol ? eta[c] : 0.0;
    const double sc = e > 0.0 ? 1.0 / e : 0.0;
#pragma unroll
    for (int rs = 0; rs < LRS; ++rs) {
      const int r = lane + 64 * rs;
      a[cs][rs] = (c < ncol && r < s) ? S[(long long)c * s + r] * sc : 0.0;
    }
  }
  double rmax = 0.0, rmin = 1e308;
  for (int j = 0; j < mu; ++j) {
    const int ow = j & 7, oc = j >> 3, jl = j & 63, js = j >> 6;
    if (wv == ow) {
      double part = 0.0, cand = 0.0;
#pragma unroll
      for (int cs = 0; cs < LCS; ++cs) {
        if (cs == oc) {
#pragma unroll
          for (int rs = 0; rs < LRS; ++rs) {
            const int r = lane + 64 * rs;
            if (r >= j) part += a[cs][rs] * a[cs][rs];
            if (rs == js) cand = a[cs][rs];
          }
        }
      }
      const double n2 = wsum(part);
      const double x1 = __shfl(cand, jl, 64);
      double beta = 0.0, tau = 0.0, scal = 0.0;
      if (n2 > 0.0) {
        const double nrm = sqrt(n2);
        beta = x1 >= 0.0 ? -nrm : nrm;
        tau = (beta - x1) / beta;
        scal = 1.0 / (x1 - beta);
      }
#pragma unroll
      for (int cs = 0; cs < LCS; ++cs) {
        if (cs == oc) {
#pragma unroll
          for (int rs = 0; rs < LRS; ++rs) {
            const int r = lane + 64 * rs;
            if (r < s) vsh[(j & 1) * (64 * LRS) + r] = r < j ? 0.0 : (r == j ? 1.0 : a[cs][rs] * scal);
            if (r == j) a[cs][rs] = beta;
            else if (r > j) a[cs][rs] = 0.0;
          }
        }
      }
      if (lane == 0) tau_sh[j & 1] = tau;
      rmax = fmax(rmax, fabs(beta));
      rmin = fmin(rmin, fabs(beta));
    }
    // one barrier per step: the reflector buffers alternate between steps
    __syncthreads();
    const double tau = tau_sh[j & 1];
    const double* vj = vsh + (j & 1) * (64 * LRS);
    double vr[LRS];
#pragma unroll
    for (int rs = 0; rs < LRS; ++rs) {
      const int r = lane + 64 * rs;
      vr[rs] = r < s ? vj[r] : 0.0;
    }
    // column dots of a group of slots first, then one interleaved butterfly
    // for the whole group (independent shuffle chains overlap).  Only the
    // slots of this wave right of column j are live (wv is wave-uniform, so
    // the tests below are scalar branches): finished columns and padding
    // skip their reductions.
    constexpr int G = (LCS + 1) / 2;
#pragma unroll
    for (int g0 = 0; g0 < LCS; g0 += G) {
      if (wv + 8 * (g0 + G - 1) <= j || wv + 8 * g0 >= ncol) continue;   // no live slot in the group
      double dt[G];
#pragma unroll
      for (int u = 0; u < G; ++u) {
        dt[u] = 0.0;
        if (g0 + u < LCS) {
#pragma unroll
          for (int rs = 0; rs < LRS; ++rs) dt[u] += vr[rs] * a[(g0 + u) < LCS ? g0 + u : 0][rs];
        }
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
        for (int u = 0; u < G; ++u) {
          const int c = wv + 8 * (g0 + u);
          if (g0 + u < LCS && c > j && c < ncol) dt[u] += __shfl_xor(dt[u], off, 64);
        }
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int c = wv + 8 * (g0 + u);
        if (g0 + u < LCS && c > j && c < ncol) {
          const double f = tau * dt[u];
#pragma unroll
          for (int rs = 0; rs < LRS; ++rs) a[(g0 + u) < LCS ? g0 + u : 0][rs] -= f * vr[rs];
        }
      }
    }
  }
  __syncthreads();
  // R and z to LDS: entry (r, c) with r <= c (r < mu)
#pragma unroll
  for (int cs = 0; cs < LCS; ++cs) {
    const int c = wv + 8 * cs;
#pragma unroll
    for (int rs = 0; rs < LRS; ++rs) {
      const int r = lane + 64 * rs;
      if (c < mu && r < mu) Rl[r + c * mu] = r <= c ? a[cs][rs] : 0.0;
      if (c == mu && r < mu) zl[r] = a[cs][rs];
    }
  }
  // |r_jj| extremes from the owner waves
  if (lane == 0) {
    rmm[2 * wv] = rmax;
    rmm[2 * wv + 1] = rmin;
  }
  __syncthreads();
}

// Same factorisation with W in global memory (any s, m); R, z to Rg / zl.
__device__ void qr_global(const double* __restrict__ S, const double* __restrict__ eta, int s, int ncol, double* W,
                          double* zl, double* sh, double* rmm) {
  const int tid = threadIdx.x, lane = tid & 63, wv = wave_id();
  const int nth = blockDim.x, nwv = nth >> 6;
  const int mu = ncol - 1;
  for (long long x = tid; x < (long long)s * ncol; x += nth) {
    const int c = (int)(x / s);
    const double e = eta[c];
    W[x] = e > 0.0 ? S[x] / e : 0.0;
  }
  __syncthreads();
  double rmax = 0.0, rmin = 1e308;
  for (int j = 0; j < mu; ++j) {
    double* wj = W + (long long)j * s;
    double part = 0.0;
    for (int r = j + tid; r < s; r += nth) part += wj[r] * wj[r];
    const double n2 = bsum(part, sh);
    const double x1 = wj[j];
    double beta = 0.0, tau = 0.0, scal = 0.0;
    if (n2 > 0.0) {
      const double nrm = sqrt(n2);
      beta = x1 >= 0.0 ? -nrm : nrm;
      tau = (beta - x1) / beta;
      scal = 1.0 / (x1 - beta);
    }
    __syncthreads();
    if (n2 > 0.0)
      for (int r = j + 1 + tid; r < s; r += nth) wj[r] *= scal;
    __syncthreads();
    if (tid == 0) wj[j] = beta;
    rmax = fmax(rmax, fabs(beta));
    rmin = fmin(rmin, fabs(beta));
    if (n2 > 0.0) {
      for (int c = j + 1 + wv; c < ncol; c += nwv) {
        double* wc = W + (long long)c * s;
        double dt = 0.0;
        for (int r = j + 1 + lane; r < s; r += 64) dt += wj[r] * wc[r];
        dt = wsum(dt) + wc[j];
        dt *= tau;
        if (lane == 0) wc[j] -= dt;
        for (int r = j + 1 + lane; r < s; r += 64) wc[r] -= dt * wj[r];
      }
    }
    __syncthreads();
  }
  for (int r = tid; r < mu; r += nth) zl[r] = W[r + (long long)mu * s];
  if (tid == 0) {
    rmm[0] = rmax;
    rmm[1] = rmin;
    for (int w = 1; w < 8; ++w) { rmm[2 * w] = 0.0; rmm[2 * w + 1] = 1e308; }
  }
  __syncthreads();
}

// ----------------------------------------------------------------- Gram matrix and Cholesky factor
// G = W^T W of the normalised sketch W = [S_0 / eta_0, ..., S_m / eta_m]
// (upper triangle, ld m+1, in the rhs's scratch region oM) on the FP64
// matrix cores: one wave per 16 x 16 tile of G, every rhs and tile in its own
// workgroup (a batch of small GEMMs).  v_mfma_f64_16x16x4f64 accumulates
// D += A B with A = W[r0 .. r0+3, ca0 .. ca0+15]^T and B = W[r0 .. r0+3,
// cb0 .. cb0+15] for r0 = 0, 4, ..., s-4: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16] and receives D[4 r + l / 16][l % 16] in its register
// r (the layout measured on gfx950).  Rows beyond s and columns beyond m are
// zero.
constexpr int GT = 16;
typedef double gram_d4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(64) k_gram(SolveDev d, DenseDev g) {
  const int q = blockIdx.x, tx = blockIdx.y, ty = blockIdx.z;
  if (ty > tx) return;   // upper tiles only
  const int lane = threadIdx.x;
  const int m1 = d.m + 1, s = d.s;
  const double* S = d.S + (long long)q * s * m1;
  const double* eta = d.eta + (long long)q * m1;
  const int ca = ty * GT + (lane & 15), cb = tx * GT + (lane & 15), kr = lane >> 4;
  const double ea = ca < m1 ? eta[ca] : 0.0, eb = cb < m1 ? eta[cb] : 0.0;
  const double ia = (ca < m1 && ea > 0.0) ? 1.0 / ea : 0.0, ib = (cb < m1 && eb > 0.0) ? 1.0 / eb : 0.0;
  const double* pa = S + (long long)(ca < m1 ? ca : 0) * s;
  const double* pb = S + (long long)(cb < m1 ? cb : 0) * s;
  gram_d4 acc = {0.0, 0.0, 0.0, 0.0};
  constexpr int U = 8;   // MFMA steps per batch of loads (32 rows)
  for (int r0 = 0; r0 < s; r0 += 4 * U) {
    double xa[U], xb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = r0 + 4 * u + kr;
      xa[u] = r < s ? pa[r] * ia : 0.0;
      xb[u] = r < s ? pb[r] * ib : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u], xb[u], acc, 0, 0, 0);
  }
  double* G = g.base + (long long)q * g.stride + g.oM;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = ty * GT + 4 * r + (lane >> 4), j = tx * GT + (lane & 15);
    if (i < m1 && j < m1 && i <= j) G[i + (long long)j * m1] = acc[r];
  }
}

// Cholesky G = R^T R of the leading n x n block of G (global, ld m1) in LDS
// (R overwrites the upper triangle, ld n), one barrier per column: step k
// updates the trailing block with the unscaled row k (G_ij -= G_ki G_kj / G_kk)
// and scales row k-1, which no step from k on reads or writes.  Fails
// (returns false, every thread) on a non-positive pivot or when the diagonal
// of R spreads more than CHOL_MAXRATIO over its first n-1 entries: then the
// squared condition number would cost accuracy and the Householder path runs.
constexpr double CHOL_MAXRATIO = 1e3;
__device__ bool cholesky_lds(const double* __restrict__ G, int m1, int n, double* R, double* rmm) {
  const int tid = threadIdx.x;
#pragma unroll 4
  for (int x = tid; x < n * n; x += LBLOCK) {
    const int i = x % n, j = x / n;
    R[x] = i <= j ? G[i + (long long)j * m1] : 0.0;
  }
  __syncthreads();
  double rmax = 0.0, rmin = 1e308, dprev = 1.0;
  for (int k = 0; k < n; ++k) {
    const double dkk = R[k + (long long)k * n];
    if (!(dkk > 0.0) || !isfinite(dkk)) return false;   // uniform: every thread read the same value
    const double rkk = sqrt(dkk);
    if (k < n - 1) {
      rmax = fmax(rmax, rkk);
      rmin = fmin(rmin, rkk);
    }
    const double inv = 1.0 / dkk;
    // trailing update: columns over waves, rows over lanes (no index division)
    for (int j = k + 1 + wave_id(); j < n; j += LBLOCK / 64) {
      const double f = R[k + j * n] * inv;
      for (int i = k + 1 + (tid & 63); i <= j; i += 64) R[i + j * n] -= R[k + i * n] * f;
    }
    if (k >= 1) {
      const double rp = sqrt(dprev);
      for (int j = k - 1 + tid; j < n; j += LBLOCK) R[k - 1 + (long long)j * n] /= rp;
    }
    dprev = dkk;
    __syncthreads();
  }
  if (tid == 0) R[n - 1 + (long long)(n - 1) * n] = sqrt(dprev);
  if (!(rmax <= CHOL_MAXRATIO * rmin)) return false;
  if (tid == 0) {
    rmm[0] = rmax;
    rmm[1] = rmin;
    for (int w = 1; w < 8; ++w) { rmm[2 * w] = 0.0; rmm[2 * w + 1] = 1e308; }
  }
  __syncthreads();
  return true;
}

// The same factorisation with G and R in global memory (R, ld n, may be any
// region of n*n doubles; G is read only), for factors too large for LDS.
// The workgroup's waves share one CU and its write-through L1, so the
// barrier per column orders the updates as in the LDS version.
__device__ bool cholesky_global(const double* __restrict__ G, int m1, int n, double* R, double* rmm) {
  const int tid = threadIdx.x;
#pragma unroll 4
  for (int x = tid; x < n * n; x += LBLOCK) {
    const int i = x % n, j = x / n;
    R[x] = i <= j ? G[i + (long long)j * m1] : 0.0;
  }
  __syncthreads();
  double rmax = 0.0, rmin = 1e308, dprev = 1.0;
  for (int k = 0; k < n; ++k) {
    const double dkk = R[k + (long long)k * n];
    if (!(dkk > 0.0) || !isfinite(dkk)) return false;   // uniform: every thread read the same value
    const double rkk = sqrt(dkk);
    if (k < n - 1) {
      rmax = fmax(rmax, rkk);
      rmin = fmin(rmin, rkk);
    }
    const double inv = 1.0 / dkk;
    for (int j = k + 1 + wave_id(); j < n; j += LBLOCK / 64) {
      const double f = R[k + (long long)j * n] * inv;
      for (int i = k + 1 + (tid & 63); i <= j; i += 64) R[i + (long long)j * n] -= R[k + (long long)i * n] * f;
    }
    if (k >= 1) {
      const double rp = sqrt(dprev);
      for (int j = k - 1 + tid; j < n; j += LBLOCK) R[k - 1 + (long long)j * n] /= rp;
    }
    dprev = dkk;
    __syncthreads();
  }
  if (tid == 0) R[n - 1 + (long long)(n - 1) * n] = sqrt(dprev);
  if (!(rmax <= CHOL_MAXRATIO * rmin)) return false;
  if (tid == 0) {
    rmm[0] = rmax;
    rmm[1] = rmin;
    for (int w = 1; w < 8; ++w) { rmm[2 * w] = 0.0; rmm[2 * w + 1] = 1e308; }
  }
  __syncthreads();
  return true;
}

__device__ inline void lsq_upper_solve(int n, const double* U, long long ldu, const double* z, double* x) {
  if (n <= 128) wave_upper_solve<2>(n, U, ldu, z, x);
  else if (n <= 256) wave_upper_solve<4>(n, U, ldu, z, x);
  else wave_upper_solve<8>(n, U, ldu, z, x);
}

// Dynamic LDS: vsh[448] + z[m+1] + (R[(m+1)^2] when the matrix fits the
// registers) + z2[m+1].
__global__ void __launch_bounds__(LBLOCK) k_lsq(SolveDev d, DenseDev g) {
  const int q = blockIdx.x;
  const int tid = threadIdx.x;
  extern __shared__ double lsh[];
  __shared__ double sh[16];
  __shared__ double rmm[16];
  __shared__ double tau_sh[2];
  const int m = d.m, m1 = d.m + 1, s = d.s;
  double* ws = g.base + (long long)q * g.stride;
  double* Hh = ws + g.oH;
  double* info = ws + g.oInfo;
  const int mu = *st_mused(d, q);
  const int brk = *st_brk(d, q);
  const double* eta = d.eta + (long long)q * m1;
  const double* H = d.H + (long long)q * m1 * m;
  const double* S = d.S + (long long)q * s * m1;
  const bool do_ls = (!brk) && mu > 0 && g.ls_mode != 2;
  const bool in_regs = s <= 64 * LRS && m + 1 <= 8 * LCS;   // as planned (m_used <= m)
  double* vsh = lsh;                    // two reflector buffers
  double* z = vsh + 2 * 64 * LRS;
  double* Rl = z + m1;
  const double* Rm = Rl;
  int ldr = mu;
  double rmax = 0.0, rmin = 1e308;
  // Cholesky of the Gram matrix (k_gram) when the sketch is well conditioned:
  // the last column of R is [z; rho], so R_m and z come out together
  bool chol = false;
  if (do_ls && in_regs) {
    chol = cholesky_lds(ws + g.oM, m1, mu + 1, Rl, rmm);
    if (chol) {
      ldr = mu + 1;
      for (int r = tid; r < mu; r += LBLOCK) z[r] = Rl[r + (long long)mu * ldr];
      __syncthreads();
    }
  }
  if (do_ls) {
    if (chol) {
      // R and z are in Rl already
    } else if (in_regs) {
      qr_registers(S, eta, s, mu + 1, vsh, Rl, z, tau_sh, rmm);
    } else {
      double* W = ws + g.oW;
      if (cholesky_global(ws + g.oM, m1, mu + 1, W, rmm)) {
        // the last column of R is [z; rho]
        Rm = W;
        ldr = mu + 1;
        for (int r = tid; r < mu; r += LBLOCK) z[r] = W[r + (long long)mu * ldr];
        __syncthreads();
      } else {
        qr_global(S, eta, s, mu + 1, W, z, sh, rmm);
        Rm = W;
        ldr = s;
      }
    }
    for (int w = 0; w < 8; ++w) {
      rmax = fmax(rmax, rmm[2 * w]);
      rmin = fmin(rmin, rmm[2 * w + 1]);
    }
    // back substitution R y = z by one wave (no barriers); R in LDS and in
    // global memory are separate call sites so that each compiles to its
    // own kind of load
    __syncthreads();
    if (tid < 64) {
      if (in_regs) lsq_upper_solve(mu, (const double*)Rl, ldr, z, z);
      else lsq_upper_solve(mu, Rm, ldr, z, z);
    }
    __syncthreads();
  } else {
    for (int x = tid; x < mu; x += LBLOCK) z[x] = 0.0;
    __syncthreads();
  }
  // H_hat = H_m + h_{m+1,m} y e_m^T (m_used x m_used, ld = mu); flat loops,
  // four loads in flight per thread
  const double hlast = (mu > 0 && !brk) ? H[(long long)(mu - 1) * m1 + mu] : 0.0;
  const int mu2 = mu * mu;
#pragma unroll 4
  for (int x = tid; x < mu2; x += LBLOCK) {
    const int r = x % mu, c = x / mu;
    double v = H[(long long)c * m1 + r];
    if (c == mu - 1) v += hlast * z[r];
    Hh[x] = v;
  }
  // R_m for the estimates (ld m_used)
  double* Rg = ws + g.oR;
  if (do_ls) {
    if (in_regs) {
#pragma unroll 4
      for (int x = tid; x < mu2; x += LBLOCK) {
        const int r = x % mu, c = x / mu;
        Rg[x] = r <= c ? Rl[r + (long long)c * ldr] : 0.0;
      }
    } else {
#pragma unroll 4
      for (int x = tid; x < mu2; x += LBLOCK) {
        const int r = x % mu, c = x / mu;
        Rg[x] = r <= c ? Rm[r + (long long)c * ldr] : 0.0;
      }
    }
  }
  if (g.nvar == 3) {
    // variant 1: H_m (no least-squares correction); variant 2: the
    // compression at order md = m_used - max(5, m_used/10)
    const long long mmf = (long long)m * m;
    double* H1 = Hh + mmf;
    double* H2 = Hh + 2 * mmf;
    int md = mu - (mu / 10 > 5 ? mu / 10 : 5);
    if (md < 1) md = 0;
#pragma unroll 4
    for (int x = tid; x < mu2; x += LBLOCK) H1[x] = H[(long long)(x / mu) * m1 + x % mu];
    double* z2 = z + m1 + (in_regs ? (long long)m1 * m1 : 0);
    if (md >= 1) {
      if (do_ls) {
        if (tid < 64) {
          // y' = R_md^{-1} R[0:md, md]: the sketched LS solution at order md
          if (in_regs) lsq_upper_solve(md, (const double*)Rl, ldr, (const double*)Rl + (long long)md * ldr, z2);
          else lsq_upper_solve(md, Rm, ldr, Rm + (long long)md * ldr, z2);
        }
      } else {
        for (int x = tid; x < md; x += LBLOCK) z2[x] = 0.0;
      }
      __syncthreads();
      const double hl2 = brk ? 0.0 : H[(long long)(md - 1) * m1 + md];
#pragma unroll 4
      for (int x = tid; x < md * md; x += LBLOCK) {
        const int r = x % md, c = x / md;
        double v = H[(long long)c * m1 + r];
        if (c == md - 1) v += hl2 * z2[r];
        H2[x] = v;
      }
    }
    if (tid == 0) info[INFO_MD] = md;
  }
  if (tid == 0) {
    info[INFO_KAPPA] = do_ls ? (rmin > 0.0 ? rmax / rmin : 1e308) : 1.0;
    info[INFO_HLAST] = hlast;
    info[INFO_BETA] = eta[0];
    info[INFO_FAIL] = 0.0;
    info[INFO_VFAIL + 1] = info[INFO_VFAIL + 2] = 0.0;
    info[INFO_LSQR_IT] = info[INFO_LSQR_RATIO] = 0.0;
  }
  double* yout = ws + g.oVec + 2 * (long long)m;
  for (int x = tid; x < mu; x += LBLOCK) yout[x] = z[x];
}

size_t lsq_lds_bytes(int s, int m) {
  const bool in_regs = s <= 64 * LRS && m + 1 <= 8 * LCS;
  return (size_t)(2 * 64 * LRS + 2 * (m + 1) + (in_regs ? (size_t)(m + 1) * (m + 1) : 0)) * 8;
}

// ----------------------------------------------------------------- polynomial
__global__ void __launch_bounds__(DBLOCK) k_fpoly(SolveDev d, DenseDev g) {
  const int q = blockIdx.x;
  const int tid = threadIdx.x;
  const DenseVariant dv = dense_variant(d, g, q, blockIdx.y);
  if (dv.dim == 0) return;
  const int m = dv.dim;
  const double* Hh = dv.H;
  double* c = dv.c;
  double* t = dv.scratch;      // scratch vector
  for (int r = tid; r < m; r += DBLOCK) c[r] = 0.0;
  __syncthreads();
  for (int j = g.ncoef - 1; j >= 0; --j) {     // Horner: c <- H_hat c + coef_j e_1
    for (int r = tid; r < m; r += DBLOCK) {
      double a = 0.0;
      for (int cc = 0; cc < m; ++cc) a += Hh[r + (long long)cc * m] * c[cc];
      t[r] = a + (r == 0 ? g.coef[j] : 0.0);
    }
    __syncthreads();
    for (int r = tid; r < m; r += DBLOCK) c[r] = t[r];
    __syncthreads();
  }
}

// ----------------------------------------------------------------- combination weights
__global__ void k_coef(SolveDev d, DenseDev g, double* cf) {
  const int q = blockIdx.x;
  const int m = d.m;
  const double* ws = g.base + (long long)q * g.stride;
  const double* c = ws + g.oVec;
  const double* eta = d.eta + (long long)q * (m + 1);
  const int mu = *st_mused(d, q);
  const double beta = eta[0];
  for (int j = threadIdx.x; j <= m; j += blockDim.x)
    cf[(long long)q * (m + 1) + j] = (j < mu && eta[j] > 0.0) ? beta * c[j] / eta[j] : 0.0;
}

hipError_t dense_set_attributes() {
  hipError_t e = hipSuccess, r;
  if ((r = hipFuncSetAttribute((const void*)k_lsq, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024)) != hipSuccess) e = r;
  if ((r = exp_set_attributes()) != hipSuccess) e = r;
  return e;
}

// ----------------------------------------------------------------- a-posteriori estimates
// With R the triangular factor of the sketched basis (||R x|| approximates
// ||V x||, Section 2.1.1), per rhs:
//   ls gate     ||R (c - c_0)|| / ||R c||     c_0 = f(H_m) e_1 (eq. (8)): how much
//                                             the least-squares column moves the result
//   convergence ||R (c - [c_{m-d}; 0])|| / ||R c||
//   rounding    u sum_j |c_j| ||R e_j|| / ||R c||   (first-order effect of
//               rounding every stored basis vector on V c)
// Without a least-squares solve (breakdown, or no LS requested) R is replaced
// by the identity.
__global__ void __launch_bounds__(256) k_estimates(SolveDev d, DenseDev g) {
  const int q = blockIdx.x, tid = threadIdx.x;
  __shared__ double sh[16];
  double* ws = g.base + (long long)q * g.stride;
  double* info = ws + g.oInfo;
  const int mu = *st_mused(d, q);
  const int brk = *st_brk(d, q);
  if (mu == 0) {
    if (tid == 0) info[INFO_GATE] = info[INFO_ROUND] = info[INFO_CONV] = 0.0;
    return;
  }
  const int md = (int)info[INFO_MD];
  const bool have_r = !brk && g.ls_mode != 2;
  const double* R = ws + g.oR;
  const DenseVariant v0 = dense_variant(d, g, q, 0), v1 = dense_variant(d, g, q, 1), v2 = dense_variant(d, g, q, 2);
  const double* c = v0.c;
  const double* c0 = v1.c;
  const double* cd = v2.c;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, sr = 0.0;
  for (int r = tid; r < mu; r += 256) {
    double w0 = 0.0, w1 = 0.0, w2 = 0.0, cn = 0.0;
    if (have_r) {
      for (int k = r; k < mu; ++k) {
        const double a = R[r + (long long)k * mu];
        w0 += a * c[k];
        w1 += a * (c[k] - c0[k]);
        w2 += a * (c[k] - (k < md ? cd[k] : 0.0));
      }
      for (int k = 0; k <= r; ++k) cn += R[k + (long long)r * mu] * R[k + (long long)r * mu];
      cn = sqrt(cn);
    } else {
      w0 = c[r];
      w1 = c[r] - c0[r];
      w2 = c[r] - (r < md ? cd[r] : 0.0);
      cn = 1.0;
    }
    s0 += w0 * w0;
    s1 += w1 * w1;
    s2 += w2 * w2;
    sr += fabs(c[r]) * cn;
  }
  s0 = bsum(s0, sh);
  s1 = bsum(s1, sh);
  s2 = bsum(s2, sh);
  sr = bsum(sr, sh);
  if (tid == 0) {
    const double n0 = sqrt(s0);
    const double inf = __builtin_huge_val();
    double gate = n0 > 0.0 ? sqrt(s1) / n0 : (s1 > 0.0 ? inf : 0.0);
    double conv = md >= 1 ? (n0 > 0.0 ? sqrt(s2) / n0 : inf) : inf;
    if (brk) gate = conv = 0.0;   // invariant subspace: the result is exact
    if (info[INFO_VFAIL + 1] != 0.0 || !isfinite(gate)) gate = inf;
    if (info[INFO_VFAIL + 2] != 0.0 || !isfinite(conv)) conv = brk ? 0.0 : inf;
    info[INFO_GATE] = gate;
    info[INFO_ROUND] = n0 > 0.0 ? g.unit_round * sr / n0 : 0.0;
    info[INFO_CONV] = conv;
  }
}

// After an LSQR refinement has rebuilt H_hat: f for the result only, the
// estimates (against the variants of the first pass) and the weights.
hipError_t fsqrt_launch(const SolveDev& d, const DenseDev& g, double* fq, hipStream_t st);

hipError_t dense_after_refine(const SolveDev& d, const DenseDev& g, double* cf, double* fq, hipStream_t st) {
  DenseDev g1 = g;
  g1.nvar = 1;
  if (g.fkind == 1)
    (void)exp_launch(d, g1, st);
  else if (g.fkind == 2) (void)fsqrt_launch(d, g1, fq, st);
  else hipLaunchKernelGGL(k_fpoly, dim3(d.nrhs, 1), dim3(DBLOCK), 0, st, d, g1);
  if (g.nvar == 3) hipLaunchKernelGGL(k_estimates, dim3(d.nrhs), dim3(256), 0, st, d, g);
  hipLaunchKernelGGL(k_coef, dim3(d.nrhs), dim3(256), 0, st, d, g, cf);
  return hipGetLastError();
}

hipError_t dense_tail(const SolveDev& d, const DenseDev& g, double* cf, double* fq, hipStream_t st) {
  if (g.ls_mode != 2) {
    // G = W^T W for the Cholesky factorisation (LDS or global memory)
    const unsigned t = (unsigned)((d.m + 1 + GT - 1) / GT);
    hipLaunchKernelGGL(k_gram, dim3(d.nrhs, t, t), dim3(64), 0, st, d, g);
  }
  hipLaunchKernelGGL(k_lsq, dim3(d.nrhs), dim3(LBLOCK), lsq_lds_bytes(d.s, d.m), st, d, g);
  const dim3 gv(d.nrhs, g.nvar);
  if (g.fkind == 1)
    (void)exp_launch(d, g, st);
  else if (g.fkind == 2) (void)fsqrt_launch(d, g, fq, st);
  else hipLaunchKernelGGL(k_fpoly, gv, dim3(DBLOCK), 0, st, d, g);
  if (g.nvar == 3) hipLaunchKernelGGL(k_estimates, dim3(d.nrhs), dim3(256), 0, st, d, g);
  hipLaunchKernelGGL(k_coef, dim3(d.nrhs), dim3(256), 0, st, d, g, cf);
  return hipGetLastError();
}

}  // namespace fab
