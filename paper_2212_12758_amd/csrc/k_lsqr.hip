// Refinement of the least-squares problem of the compression (eq. (7)) by
// LSQR preconditioned with the triangular factor R of the sketched basis
// (Blendenpik, the preconditioner Section 3.1.1 uses):
//     min_z || V_m R^{-1} z - v_{m+1} ||_2,   started from z = 0,   y = R^{-1} z.
// LSQR (Paige & Saunders, ACM TOMS 8 (1982)) in its standard form: the
// operator M = V_m R^{-1} is applied as M p = sum_j (p_j / eta_j) u_j with
// p = R^{-1} v (a pass over the basis), and M^T u = R^{-T} diag(1/eta) U^T u.
//
// One iteration = k_lsqr_pass (stream the basis once: form the new n-vector
// u~ <- M v - (alpha/beta) u~ and, on the same tile, its dots with every
// basis vector and its norm, as per-block partials) + k_lsqr_step (one
// workgroup per rhs: reduce the partials in a fixed order, the triangular
// solves with R and R^T, the LSQR recurrences, the stopping test and the
// coefficients of the next pass).  The launch sequence has a fixed length;
// once every rhs has stopped the remaining launches return immediately.
//
// Stopping test: Paige & Saunders' second criterion, ||M^T r|| <= atol
// ||M|| ||r|| (the iterate then solves a least-squares problem whose matrix
// is within a relative atol of M), with ||r_k|| = phibar_{k+1},
// ||M^T r_k|| = phibar_{k+1} alpha_{k+1} |c_k| and their Frobenius-norm
// estimate ||M||_F^2 ~ sum (alpha_k^2 + beta_{k+1}^2), so the test reads
// alpha_{k+1} |c_k| / ||M||_F <= atol.  An iteration limit reached before
// that is recorded (INFO_LSQR_LIMIT).
#include "k_basis.h"

namespace fab {

namespace {

// per-rhs state, stride lsqr_state_stride(m) doubles:
//   [0, m1) v   [m1, 2m1) w   [2m1, 3m1) x   [3m1, 4m1) pass coefficients
//   [4m1, 5m1) scratch   then scalars at 5m1 + k
// LS_RATIO: the Paige-Saunders measure alpha |c| / ||M||_F of the last
// iteration; LS_ANORM2: the running ||M||_F^2 estimate; LS_LIMIT: 1 when the
// iteration limit stopped the refinement before the test was met.
enum { LS_A = 0, LS_ALPHA, LS_BETA, LS_RHOBAR, LS_PHIBAR, LS_DONE, LS_ITERS, LS_RATIO, LS_ANORM2, LS_LIMIT,
       LS_NSCAL = 16 };

// Solve U^T x = z (U upper triangular, column-major, leading dimension ldu)
// by one wave: forward substitution with rows in registers.
template <int R>
__device__ void wave_upper_t_solve(int n, const double* U, long long ldu, const double* z, double* x) {
  const int lane = threadIdx.x & 63;
  double y[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int r = lane + 64 * u;
    y[u] = r < n ? z[r] : 0.0;
  }
  for (int j = 0; j < n; ++j) {
    const int uj = j >> 6;
    double src = y[0];
#pragma unroll
    for (int u = 1; u < R; ++u)
      if (uj == u) src = y[u];
    const double ujj = U[j + (long long)j * ldu];
    const double xj = ujj != 0.0 ? readlane_d(src, j & 63) / ujj : 0.0;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int r = lane + 64 * u;
      if (r == j) y[u] = xj;
      else if (r > j && r < n) y[u] -= U[j + (long long)r * ldu] * xj;
    }
  }
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int r = lane + 64 * u;
    if (r < n) x[r] = y[u];
  }
}

__device__ void upper_solve_any(int n, const double* U, long long ldu, const double* z, double* x) {
  if (n <= 128) wave_upper_solve<2>(n, U, ldu, z, x);
  else if (n <= 256) wave_upper_solve<4>(n, U, ldu, z, x);
  else wave_upper_solve<8>(n, U, ldu, z, x);
}
__device__ void upper_t_solve_any(int n, const double* U, long long ldu, const double* z, double* x) {
  if (n <= 128) wave_upper_t_solve<2>(n, U, ldu, z, x);
  else if (n <= 256) wave_upper_t_solve<4>(n, U, ldu, z, x);
  else wave_upper_t_solve<8>(n, U, ldu, z, x);
}

__device__ inline double bsum256(double v, double* sh) {
  v = wave_sum_all(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  const double t = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return t;
}

}  // namespace

size_t lsqr_state_stride(int m) { return (size_t)5 * (m + 1) + LS_NSCAL; }
size_t lsqr_pass_lds(int m, int nrhs) { return (size_t)4 * nrhs * (m + 1) * 8; }
size_t lsqr_pass1_lds(int m, int ch, int esize) {
  return ((size_t)m * (ch + 1) * esize + 7) / 8 * 8 + (size_t)ch * 8 + (size_t)m * 8;
}
// Chunk of the one-read pass (0: the two-read pass): one rhs, m + 1 <= 256,
// and the staged tile within 80 KB, so that two blocks share a CU.
int lsqr_pass1_chunk(int m, int nrhs, int esize) {
  if (nrhs != 1 || m + 1 > 256) return 0;
  if (lsqr_pass1_lds(m, 128, esize) <= 80 * 1024) return 128;
  if (lsqr_pass1_lds(m, 64, esize) <= 80 * 1024) return 64;
  return 0;
}

// Stream the basis once.  first: u~ = u_m / eta_m (the right-hand side
// v_{m+1}); else u~ <- sum_j cf_j u_j - a u~.  Partials per block and rhs:
// the dots u_j^T u~ (j < m) and ||u~||^2 (slot m).
template <typename T, bool NR1>
__global__ void __launch_bounds__(256) k_lsqr_pass(SolveDev d, LsqrDev L, int first) {
  if (*L.alldone) return;
  extern __shared__ double acc[];   // [wave][rhs][m+1]
  const int tid = threadIdx.x, lane = tid & 63, wv = wave_id();
  const int nr = d.nrhs, m = d.m, m1 = m + 1;
  const T* __restrict__ V = (const T*)d.V;
  const long long nel = (long long)d.n * nr;
  for (int x = tid; x < 4 * nr * m1; x += 256) acc[x] = 0.0;
  __syncthreads();
  int rq[EPT];   // rhs of each element (0 with one rhs: the coefficients are then uniform)
#pragma unroll
  for (int j = 0; j < EPT; ++j) rq[j] = NR1 ? 0 : (tid * EPT + j) & (nr - 1);
  for (long long e = ((long long)blockIdx.x * 256 + tid) * EPT; e - (long long)tid * EPT < nel;
       e += (long long)gridDim.x * 256 * EPT) {
    const bool live = e < nel;
    double un[EPT];
    if (live) {
      if (first) {
        get8(V + (long long)m * d.ldv, e, nel, un);
#pragma unroll
        for (int j = 0; j < EPT; ++j) un[j] /= d.eta[(long long)rq[j] * m1 + m];
      } else {
        double old[EPT];
        get8(L.u, e, nel, old);
#pragma unroll
        for (int j = 0; j < EPT; ++j) un[j] = -L.st[(long long)rq[j] * L.stride + 5 * m1 + LS_A] * old[j];
        int jv = 0;
        if (e + EPT <= nel) {
          for (; jv + 4 <= m; jv += 4) {
            double v[4][EPT];
#pragma unroll
            for (int u = 0; u < 4; ++u) load8(V + (long long)(jv + u) * d.ldv + e, v[u]);
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
              for (int j = 0; j < EPT; ++j) un[j] += L.st[(long long)rq[j] * L.stride + 3 * m1 + jv + u] * v[u][j];
          }
        }
        for (; jv < m; ++jv) {
          double v[EPT];
          get8(V + (long long)jv * d.ldv, e, nel, v);
#pragma unroll
          for (int j = 0; j < EPT; ++j) un[j] += L.st[(long long)rq[j] * L.stride + 3 * m1 + jv] * v[j];
        }
      }
      if (e + EPT <= nel) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          double2 o;
          o.x = un[2 * h];
          o.y = un[2 * h + 1];
          *reinterpret_cast<double2*>(L.u + e + 2 * h) = o;
        }
      } else {
        for (int j = 0; j < EPT; ++j)
          if (e + j < nel) L.u[e + j] = un[j];
      }
    } else {
#pragma unroll
      for (int j = 0; j < EPT; ++j) un[j] = 0.0;
    }
    // dots with the basis and the norm, reduced per wave into LDS slots
    // (full chunks: four basis vectors per round, loads issued together)
    const bool full = e + EPT <= nel;
    for (int jv0 = 0; jv0 <= m; jv0 += 4) {
      double v[4][EPT];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int jv = jv0 + u;
        if (jv < m && full) {
          load8(V + (long long)jv * d.ldv + e, v[u]);
        } else if (jv < m && live) {
          get8(V + (long long)jv * d.ldv, e, nel, v[u]);
        } else {
#pragma unroll
          for (int j = 0; j < EPT; ++j) v[u][j] = jv == m ? un[j] : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int jv = jv0 + u;
        if (jv > m) break;
        for (int q = 0; q < nr; ++q) {
          double p = 0.0;
#pragma unroll
          for (int j = 0; j < EPT; ++j)
            if (rq[j] == q) p += v[u][j] * un[j];
          p = wave_sum_all(p);
          if (lane == 0) acc[(wv * nr + q) * m1 + jv] += p;
        }
      }
    }
  }
  __syncthreads();
  for (int x = tid; x < nr * m1; x += 256)
    L.part[(long long)blockIdx.x * nr * m1 + x] = (acc[x] + acc[nr * m1 + x]) + (acc[2 * nr * m1 + x] + acc[3 * nr * m1 + x]);
}

// One-read pass for one rhs: each chunk of CH elements of every basis
// vector u_0..u_{m-1} is staged once in LDS (row j at j * (CH + 1): odd
// stride, so the column reads of the dots spread over the banks); thread t
// forms u~ on element t from the staged values (the same operations, in the
// same order, as k_lsqr_pass), then thread j accumulates u_j^T u~ over the
// chunk (thread m: ||u~||^2), so the basis is read from memory once per pass
// instead of twice.  Per-block partials in the same layout as k_lsqr_pass.
// Requires m + 1 <= 256 and the LDS of lsqr_pass1_lds.
template <typename T, int CH>
__global__ void __launch_bounds__(256) k_lsqr_pass1(SolveDev d, LsqrDev L, int first) {
  if (*L.alldone) return;
  extern __shared__ double p1lds[];
  constexpr int LD = CH + 1;
  constexpr int VW = 16 / sizeof(T);   // elements per 16-byte load
  const int tid = threadIdx.x;
  const int m = d.m, m1 = m + 1;
  T* Vs = reinterpret_cast<T*>(p1lds);                                    // [m][LD]
  double* us = p1lds + ((long long)m * LD * (long long)sizeof(T) + 7) / 8;   // [CH]
  double* cfs = us + CH;                                                  // [m]
  const T* __restrict__ V = (const T*)d.V;
  const long long nel = d.n;
  const double a = first ? 0.0 : L.st[5 * m1 + LS_A];
  const double em = d.eta[m];
  for (int j = tid; j < m; j += 256) cfs[j] = first ? 0.0 : L.st[3 * m1 + j];
  double dacc = 0.0;
  const int items = m * (CH / VW);   // 16-byte pieces of the staged tile
  const long long nchunk = (nel + CH - 1) / CH;
  for (long long c = blockIdx.x; c < nchunk; c += gridDim.x) {
    const long long e0 = c * CH;
    __syncthreads();   // the previous chunk's dots are done with Vs and us
    for (int x0 = tid; x0 < items; x0 += 256 * 8) {
      T w[8][VW];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int x = x0 + 256 * r;
        const int j = x / (CH / VW), t = (x - j * (CH / VW)) * VW;
        const long long e = e0 + t;
        if (x < items && e + VW <= nel) {
          const T* src = V + (long long)j * d.ldv + e;
          if constexpr (VW == 4) {
            const float4 f = *reinterpret_cast<const float4*>(src);
            w[r][0] = f.x; w[r][1] = f.y; w[r][2] = f.z; w[r][3] = f.w;
          } else {
            const double2 f = *reinterpret_cast<const double2*>(src);
            w[r][0] = f.x; w[r][1] = f.y;
          }
        } else {
#pragma unroll
          for (int v = 0; v < VW; ++v) w[r][v] = (x < items && e + v < nel) ? V[(long long)j * d.ldv + e + v] : (T)0;
        }
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int x = x0 + 256 * r;
        if (x < items) {
          const int j = x / (CH / VW), t = (x - j * (CH / VW)) * VW;
#pragma unroll
          for (int v = 0; v < VW; ++v) Vs[j * LD + t + v] = w[r][v];
        }
      }
    }
    __syncthreads();
    if (tid < CH) {
      const long long e = e0 + tid;
      double un = 0.0;
      if (e < nel) {
        if (first) {
          un = (double)V[(long long)m * d.ldv + e] / em;
        } else {
          un = -a * L.u[e];
          for (int j = 0; j < m; ++j) un += cfs[j] * (double)Vs[j * LD + tid];
        }
        L.u[e] = un;
      }
      us[tid] = un;
    }
    __syncthreads();
    if (tid < m) {
      const T* row = Vs + tid * LD;
      double sdot = 0.0;
      for (int t = 0; t < CH; ++t) sdot += (double)row[t] * us[t];
      dacc += sdot;
    } else if (tid == m) {
      double sdot = 0.0;
      for (int t = 0; t < CH; ++t) sdot += us[t] * us[t];
      dacc += sdot;
    }
  }
  if (tid < m1) L.part[(long long)blockIdx.x * m1 + tid] = dacc;
}

// X = R_m^{-1} and X^T for the LSQR steps, computed once per refinement, so
// that each step applies the preconditioner as two triangular matrix-vector
// products spread over the block instead of two sequential substitutions on
// one wave.  Column j of X solves R x = e_j: x_i /= r_ii, then
// x[0..i-1] -= R[0..i-1, i] x_i for i = j, j-1, .., 0 (column-oriented back
// substitution), one wave per column, each lane holding rows lane + 64 u, the
// next column of R loaded while the current one is applied.  LSQR then runs
// on M = V_m X, and the refined y = X z, so the iterates and the result use
// the same operator.
// RINV_RMAX rows per lane: m <= 64 RINV_RMAX (instances for 2, 4 and 8, so
// that a step touches only the registers its rows need)
template <int RINV_RMAX>
__global__ void __launch_bounds__(256) k_lsqr_rinv(SolveDev d, DenseDev g, LsqrDev L) {
  const int q = blockIdx.x, lane = threadIdx.x & 63;
  const int mu = d.status[4 + 2 * q];
  const int brk = d.status[5 + 2 * q];
  if (brk || mu == 0 || g.ls_mode == 2) return;
  const int j = blockIdx.y * 4 + wave_id();
  if (j >= mu) return;   // (no block barrier below)
  const int m = d.m;
  const double* R = g.base + (long long)q * g.stride + g.oR;   // ld mu
  double* X = L.rinv + (long long)q * 2 * m * m;
  double* XT = X + (long long)m * m;
  double x[RINV_RMAX], rc[RINV_RMAX], rn[RINV_RMAX];
#pragma unroll
  for (int u = 0; u < RINV_RMAX; ++u) {
    const int r = lane + 64 * u;
    x[u] = r == j ? 1.0 : 0.0;
    rc[u] = r <= j ? R[r + (long long)j * mu] : 0.0;
  }
  for (int i = j; i >= 0; --i) {
#pragma unroll
    for (int u = 0; u < RINV_RMAX; ++u) {
      const int r = lane + 64 * u;
      rn[u] = (i > 0 && r <= i - 1) ? R[r + (long long)(i - 1) * mu] : 0.0;
    }
    const int ui = i >> 6, li = i & 63;
    double xs = x[0], rs = rc[0];
#pragma unroll
    for (int u = 1; u < RINV_RMAX; ++u)
      if (ui == u) { xs = x[u]; rs = rc[u]; }
    const double xi = readlane_d(xs, li) / readlane_d(rs, li);
#pragma unroll
    for (int u = 0; u < RINV_RMAX; ++u) {
      const int r = lane + 64 * u;
      if (r == i) x[u] = xi;
      else if (r < i) x[u] -= rc[u] * xi;
    }
#pragma unroll
    for (int u = 0; u < RINV_RMAX; ++u) rc[u] = rn[u];
  }
#pragma unroll
  for (int u = 0; u < RINV_RMAX; ++u) {
    const int r = lane + 64 * u;
    if (r < mu) {
      X[r + (long long)j * mu] = r <= j ? x[u] : 0.0;
      XT[j + (long long)r * mu] = r <= j ? x[u] : 0.0;
    }
  }
}

// Entries [ka, kb) of row i of A (column-major, ld mu) times c (in LDS): 16
// entries of the row loaded per round before they are used, eight partial
// sums in a fixed order.
__device__ inline double rinv_row(const double* __restrict__ A, int mu, int i, const double* cs, int ka, int kb) {
  double s[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) s[u] = 0.0;
  int k = ka;
  for (; k + 16 <= kb; k += 16) {
    double a[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) a[u] = A[i + (long long)(k + u) * mu];
#pragma unroll
    for (int u = 0; u < 16; ++u) s[u & 7] += a[u] * cs[k + u];
  }
  for (; k < kb; ++k) s[0] += A[i + (long long)k * mu] * cs[k];
  return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// out = X^T c (lower: the transpose, stored) or X c, X upper triangular: row
// i sums over k <= i (lower) or k >= i.  c is staged in LDS first; with at
// most 128 rows two threads share a row (the two halves of its range, added
// in that order).  Every thread of the block calls it (it has barriers);
// out must not alias c.
__device__ inline void rinv_apply(int mu, const double* __restrict__ A, bool lower, const double* c, double* out) {
  __shared__ double cs[512];
  __shared__ double hsum[128];
  const int tid = threadIdx.x;
  for (int k = tid; k < mu; k += 256) cs[k] = c[k];
  __syncthreads();
  if (mu <= 128) {
    const int i = tid & 127, h = tid >> 7;
    double part = 0.0;
    if (i < mu) {
      const int k0 = lower ? 0 : i, k1 = lower ? i + 1 : mu;
      const int mid = k0 + (k1 - k0) / 2;
      part = h ? rinv_row(A, mu, i, cs, mid, k1) : rinv_row(A, mu, i, cs, k0, mid);
    }
    if (h) hsum[i] = part;
    __syncthreads();
    if (!h && i < mu) out[i] = part + hsum[i];
  } else {
    for (int i = tid; i < mu; i += 256)
      out[i] = rinv_row(A, mu, i, cs, lower ? 0 : i, lower ? i + 1 : mu);
  }
  __syncthreads();
}

// One LSQR step per rhs (first: the initialisation).  The preconditioner is
// applied through X = R_m^{-1} (k_lsqr_rinv).
__global__ void __launch_bounds__(256) k_lsqr_step(SolveDev d, DenseDev g, LsqrDev L, int first) {
  if (*L.alldone) return;
  const int q = blockIdx.x, tid = threadIdx.x;
  __shared__ double sh[8];
  const int nr = d.nrhs, m = d.m, m1 = m + 1;
  double* st = L.st + (long long)q * L.stride;
  double* v = st;
  double* w = st + m1;
  double* x = st + 2 * m1;
  double* cf = st + 3 * m1;
  double* tmp = st + 4 * m1;
  double* sc = st + 5 * m1;
  const int mu = d.status[4 + 2 * q];
  const int brk = d.status[5 + 2 * q];
  const double* eta = d.eta + (long long)q * m1;
  if (first) {
    if (tid == 0) {
      sc[LS_DONE] = (brk || mu == 0 || g.ls_mode == 2) ? 1.0 : 0.0;
      sc[LS_ITERS] = 0.0;
      sc[LS_RATIO] = 0.0;
      sc[LS_ANORM2] = 0.0;
      sc[LS_LIMIT] = 0.0;
    }
    for (int j = tid; j < m1; j += 256) x[j] = 0.0;
    __syncthreads();
  }
  if (sc[LS_DONE] != 0.0) {
    if (nr == 1 && tid == 0) *L.alldone = 1;   // one rhs: no separate all-done launch
    return;
  }
  // reduce the pass partials in a fixed order: thread (group g, slot j)
  // sums blocks [g nb / G, (g+1) nb / G) in order, up to 64 loads in flight,
  // then the G group sums are added in order
  {
    __shared__ double gsum[256];
    const int ns = mu + 1;
    const int G = ns >= 256 ? 1 : 256 / ns;
    for (int j0 = 0; j0 < ns; j0 += 256 / G) {
      const int j = j0 + tid % (256 / G), grp = tid / (256 / G);
      double a = 0.0;
      if (j < ns && grp < G) {
        const int slot = j < mu ? j : m;
        const int b0 = (int)((long long)grp * L.nblk / G), b1 = (int)((long long)(grp + 1) * L.nblk / G);
        // 64 loads in flight (the sum itself stays in block order)
        int b = b0;
        for (; b + 64 <= b1; b += 64) {
          double t[64];
#pragma unroll
          for (int u = 0; u < 64; ++u) t[u] = L.part[((long long)(b + u) * nr + q) * m1 + slot];
#pragma unroll
          for (int u = 0; u < 64; ++u) a += t[u];
        }
        for (; b + 8 <= b1; b += 8) {
          double t[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) t[u] = L.part[((long long)(b + u) * nr + q) * m1 + slot];
#pragma unroll
          for (int u = 0; u < 8; ++u) a += t[u];
        }
        for (; b < b1; ++b) a += L.part[((long long)b * nr + q) * m1 + slot];
      }
      gsum[tid] = a;
      __syncthreads();
      if (tid < 256 / G && j0 + tid < ns) {
        double t = 0.0;
        for (int gg = 0; gg < G; ++gg) t += gsum[gg * (256 / G) + tid];
        tmp[j0 + tid] = t;
      }
      __syncthreads();
    }
  }
  const double beta = sqrt(tmp[mu]);
  // s = R^{-T} (d / eta) / beta  ->  cf (scratch)
  for (int j = tid; j < mu; j += 256) cf[j] = beta > 0.0 ? tmp[j] / (eta[j] * beta) : 0.0;
  __syncthreads();
  const double* Xq = L.rinv + (long long)q * 2 * m * m;   // X = R^{-1}, then X^T
  rinv_apply(mu, Xq + (long long)m * m, true, cf, tmp);    // tmp = R^{-T} cf
  __syncthreads();
  // alpha v = s - beta v_old
  double p2 = 0.0;
  for (int j = tid; j < mu; j += 256) {
    const double t = first ? tmp[j] : tmp[j] - beta * v[j];
    tmp[j] = t;
    p2 += t * t;
  }
  const double alpha = sqrt(bsum256(p2, sh));
  for (int j = tid; j < mu; j += 256) v[j] = alpha > 0.0 ? tmp[j] / alpha : 0.0;
  __syncthreads();
  if (first) {
    for (int j = tid; j < mu; j += 256) w[j] = v[j];
    if (tid == 0) {
      sc[LS_PHIBAR] = beta;
      sc[LS_RHOBAR] = alpha;
      sc[LS_ALPHA] = alpha;
      if (!(beta > 0.0) || !(alpha > 0.0)) sc[LS_DONE] = 1.0;   // y = 0 solves it
    }
  } else {
    const double rhobar = sc[LS_RHOBAR], phibar = sc[LS_PHIBAR];
    const double rho = sqrt(rhobar * rhobar + beta * beta);
    const double c = rho > 0.0 ? rhobar / rho : 1.0, s = rho > 0.0 ? beta / rho : 0.0;
    const double theta = s * alpha, phi = c * phibar;
    const double step = rho > 0.0 ? phi / rho : 0.0;
    for (int j = tid; j < mu; j += 256) {
      x[j] += step * w[j];
      w[j] = v[j] - (rho > 0.0 ? theta / rho : 0.0) * w[j];
    }
    __syncthreads();
    if (tid == 0) {
      const double alpha_old = sc[LS_ALPHA];
      const double anorm2 = sc[LS_ANORM2] + alpha_old * alpha_old + beta * beta;
      sc[LS_ANORM2] = anorm2;
      sc[LS_ALPHA] = alpha;
      sc[LS_RHOBAR] = -c * alpha;
      sc[LS_PHIBAR] = s * phibar;
      sc[LS_ITERS] += 1.0;
      // ||M^T r|| / (||M||_F ||r||)
      const double ps = anorm2 > 0.0 ? alpha * fabs(c) / sqrt(anorm2) : 0.0;
      sc[LS_RATIO] = ps;
      const bool met = ps <= L.tol || !(alpha > 0.0) || !(beta > 0.0);
      if (met) {
        sc[LS_DONE] = 1.0;
      } else if (sc[LS_ITERS] >= L.maxit) {
        sc[LS_DONE] = 1.0;
        sc[LS_LIMIT] = 1.0;
      }
    }
  }
  if (nr == 1 && tid == 0 && sc[LS_DONE] != 0.0) *L.alldone = 1;
  __syncthreads();
  // coefficients of the next pass: cf = R^{-1} v / eta, a = alpha / beta
  rinv_apply(mu, Xq, false, v, tmp);
  __syncthreads();
  for (int j = tid; j < m; j += 256) cf[j] = j < mu ? tmp[j] / eta[j] : 0.0;
  if (tid == 0) sc[LS_A] = beta > 0.0 ? alpha / beta : 0.0;
}

// All rhs stopped?  (one thread; keeps the remaining launches empty.  With
// one rhs the step kernel sets the flag itself and this is not launched.)
__global__ void k_lsqr_alldone(SolveDev d, LsqrDev L) {
  if (threadIdx.x != 0 || *L.alldone) return;
  const int m1 = d.m + 1;
  int all = 1;
  for (int q = 0; q < d.nrhs; ++q) all &= L.st[(long long)q * L.stride + 5 * m1 + LS_DONE] != 0.0;
  *L.alldone = all;
}

// y = R^{-1} z, H_hat = H_m + h_{m+1,m} y e_m^T, iteration count to the info block.
__global__ void __launch_bounds__(256) k_lsqr_finish(SolveDev d, DenseDev g, LsqrDev L) {
  const int q = blockIdx.x, tid = threadIdx.x;
  const int m = d.m, m1 = m + 1;
  double* ws = g.base + (long long)q * g.stride;
  const double* st = L.st + (long long)q * L.stride;
  const double* sc = st + 5 * m1;
  const int mu = d.status[4 + 2 * q];
  const int brk = d.status[5 + 2 * q];
  double* info = ws + g.oInfo;
  if (tid == 0) {
    info[INFO_LSQR_IT] = sc[LS_ITERS];
    info[INFO_LSQR_RATIO] = sc[LS_RATIO];
    info[INFO_LSQR_LIMIT] = sc[LS_LIMIT];
  }
  if (brk || mu == 0 || g.ls_mode == 2) return;
  __shared__ double y[512];
  rinv_apply(mu, L.rinv + (long long)q * 2 * m * m, false, st + 2 * m1, y);   // y = X z
  __syncthreads();
  double* yout = ws + g.oVec + 2 * (long long)m;
  for (int j = tid; j < mu; j += 256) yout[j] = y[j];
  const double* H = d.H + (long long)q * m1 * m;
  const double hlast = H[(long long)(mu - 1) * m1 + mu];
  double* Hh = ws + g.oH;
  for (int c = wave_id(); c < mu; c += 4)
    for (int r = tid & 63; r < mu; r += 64) {
      double val = H[(long long)c * m1 + r];
      if (c == mu - 1) val += hlast * y[r];
      Hh[r + (long long)c * mu] = val;
    }
}

// ------------------------------------------------------------------ exact least squares from the Gram matrix
// For a well-conditioned basis (sketched Gram-Schmidt, whitened) the least
// squares of eq. (7) are solved exactly through the normal equations: one
// pass over the stored vectors forms G = U^T U (FP64 accumulation, one right-
// hand side, m + 1 <= GR_MAXC), then with D = diag(eta), G~ = D^{-1} G D^{-1},
// G~_m = R^T R (Cholesky) and R^T R y = G~[:m, m].  The error is about
// kappa(V)^2 u (u the FP64 unit roundoff); the factorisation reports failure
// (the caller then runs LSQR) on a non-positive pivot, a diagonal spread of R
// above GR_MAXRATIO, or an estimated kappa_1(R) above `maxcond` =
// min(GR_MAXCOND, sqrt(tol / (10 u))), so that kappa^2 u <= tol / 10.
constexpr int GR_TILE = 16, GR_T = 8, GR_MAXC = GR_T * GR_TILE;   // m + 1 <= 128
constexpr int GR_NT = GR_T * (GR_T + 1) / 2;                      // upper 16 x 16 tiles
constexpr int GR_RCH = 32;                                          // rows per staged chunk
constexpr int GR_BLOCKS = 240;
constexpr double GR_MAXRATIO = 1e4;
constexpr double GR_MAXCOND = 1e4;   // largest accepted kappa_1(R) estimate

// kappa_1(R) = ||R||_1 ||R^{-1}||_1 of an upper triangular R (n <= 128) by
// one wave: ||R||_1 exactly, ||R^{-1}||_1 by Hager's 1-norm estimator (Hager
// 1984, in Higham's formulation): x = ones/n; y = R^{-1} x, z = R^{-T} sign(y);
// stop when ||z||_inf <= z^T x or ||y||_1 stops growing, else x = e_j at the
// largest |z_j|; at most 5 rounds.  The estimate is a lower bound, in practice
// within a small factor.  xv, zv: LDS vectors of n doubles.  A small diagonal
// spread does not imply a small condition number (the columns of a truncated
// Krylov basis can be nearly dependent while every pivot stays O(1)), hence
// this check beside the spread test.
__device__ double wave_kappa1_upper(int n, const double* R, long long ld, double* xv, double* zv) {
  const int lane = threadIdx.x & 63;
  double rn = 0.0;
  for (int j = lane; j < n; j += 64) {
    double c = 0.0;
    for (int i = 0; i <= j; ++i) c += fabs(R[i + (long long)j * ld]);
    rn = fmax(rn, c);
  }
  for (int off = 32; off >= 1; off >>= 1) rn = fmax(rn, __shfl_xor(rn, off, 64));
  for (int i = lane; i < n; i += 64) xv[i] = 1.0 / n;
  double est = 0.0;
  int jprev = -1;
  for (int it = 0; it < 5; ++it) {
    upper_solve_any(n, R, ld, xv, xv);   // y = R^{-1} x
    double s = 0.0;
    for (int i = lane; i < n; i += 64) {
      s += fabs(xv[i]);
      zv[i] = xv[i] >= 0.0 ? 1.0 : -1.0;
    }
    const double e = wave_sum_all(s);
    if (it > 0 && !(e > est)) break;
    est = e;
    upper_t_solve_any(n, R, ld, zv, zv);   // z = R^{-T} sign(y)
    double bv = -1.0, zs = 0.0;
    int bi = 0;
    for (int i = lane; i < n; i += 64) {
      const double a = fabs(zv[i]);
      zs += zv[i];
      if (a > bv) {
        bv = a;
        bi = i;
      }
    }
    for (int off = 32; off >= 1; off >>= 1) {
      const double ov = __shfl_xor(bv, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    const double zx = jprev < 0 ? wave_sum_all(zs) / n : zv[jprev];
    if (!(bv > zx)) break;
    jprev = bi;
    for (int i = lane; i < n; i += 64) xv[i] = i == bi ? 1.0 : 0.0;
  }
  return rn * est;
}

// Per-block partial sums of the upper tiles of U^T U: part[blk][tile][entry].
template <typename T>
__global__ void __launch_bounds__(256) k_vgram(SolveDev d, double* __restrict__ part) {
  __shared__ double ul[GR_RCH][GR_MAXC + 1];
  const int tid = threadIdx.x, a0 = tid & (GR_TILE - 1), b0 = tid >> 4;
  const int m1 = d.m + 1;
  const long long n = d.n;
  const T* __restrict__ V = (const T*)d.V;
  double acc[GR_NT];
#pragma unroll
  for (int t = 0; t < GR_NT; ++t) acc[t] = 0.0;
  for (long long r0 = (long long)blockIdx.x * GR_RCH; r0 < n; r0 += (long long)gridDim.x * GR_RCH) {
    // stage rows r0 .. r0+31 of every column (column-contiguous loads), 16 in flight
    double t16[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int x = tid + 256 * u, c = x >> 5, rr = x & 31;
      const long long r = r0 + rr;
      t16[u] = (c < m1 && r < n) ? (double)V[(long long)c * d.ldv + r] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int x = tid + 256 * u;
      ul[x & 31][x >> 5] = t16[u];
    }
    __syncthreads();
    for (int rr = 0; rr < GR_RCH; ++rr) {
      double xa[GR_T], xb[GR_T];
#pragma unroll
      for (int t = 0; t < GR_T; ++t) {
        xa[t] = ul[rr][GR_TILE * t + a0];
        xb[t] = ul[rr][GR_TILE * t + b0];
      }
      int idx = 0;
#pragma unroll
      for (int ti = 0; ti < GR_T; ++ti)
#pragma unroll
        for (int tj = ti; tj < GR_T; ++tj) acc[idx++] += xa[ti] * xb[tj];
    }
    __syncthreads();
  }
  double* out = part + (long long)blockIdx.x * GR_NT * 256;
#pragma unroll
  for (int t = 0; t < GR_NT; ++t) out[t * 256 + tid] = acc[t];
}

// Fixed-order sum over the blocks, scaled to G~ = D^{-1} G D^{-1}; G~ (ld m1,
// upper triangle) goes to the rhs's scratch region.  One workgroup per tile.
__global__ void __launch_bounds__(256) k_vgram_reduce(SolveDev d, DenseDev g, const double* __restrict__ part,
                                                      int nb) {
  const int t = blockIdx.x, tid = threadIdx.x, a0 = tid & (GR_TILE - 1), b0 = tid >> 4;
  int ti = 0, tj = 0, idx = 0;
  for (int i = 0; i < GR_T; ++i)
    for (int j = i; j < GR_T; ++j) {
      if (idx == t) { ti = i; tj = j; }
      ++idx;
    }
  const int a = GR_TILE * ti + a0, b = GR_TILE * tj + b0;
  const int m1 = d.m + 1;
  double s = 0.0;
  int blk = 0;
  for (; blk + 8 <= nb; blk += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[((long long)(blk + u) * GR_NT + t) * 256 + tid];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; blk < nb; ++blk) s += part[((long long)blk * GR_NT + t) * 256 + tid];
  if (a < m1 && b < m1 && a <= b) {
    const double ea = d.eta[a], eb = d.eta[b];
    g.base[g.oM + a + (long long)b * m1] = (ea > 0.0 && eb > 0.0) ? s / (ea * eb) : 0.0;
  }
}

// Cholesky of G~_m, y from the normal equations, H_hat; *fail = 1 when the
// factorisation is not usable (the caller then refines by LSQR instead).
__global__ void __launch_bounds__(512) k_vgram_solve(SolveDev d, DenseDev g, int* fail, double maxcond) {
  extern __shared__ double R[];   // mu x mu, ld mu
  __shared__ double rhs[GR_MAXC], y[GR_MAXC];
  const int tid = threadIdx.x;
  const int m = d.m, m1 = m + 1;
  double* ws = g.base;
  const double* G = ws + g.oM;
  const int mu = d.status[4];
  const int brk = d.status[5];
  double* info = ws + g.oInfo;
  if (tid == 0) {
    *fail = 0;
    info[INFO_LSQR_IT] = 0.0;
    info[INFO_LSQR_RATIO] = 0.0;
    info[INFO_LSQR_LIMIT] = 0.0;
  }
  if (brk || mu == 0 || g.ls_mode == 2) return;
  for (int x = tid; x < mu * mu; x += 512) {
    const int i = x % mu, j = x / mu;
    R[x] = i <= j ? G[i + (long long)j * m1] : 0.0;
  }
  for (int i = tid; i < mu; i += 512) rhs[i] = G[i + (long long)mu * m1];
  __syncthreads();
  double rmax = 0.0, rmin = 1e308, dprev = 1.0;
  for (int k = 0; k < mu; ++k) {
    const double dkk = R[k + k * mu];
    if (!(dkk > 0.0) || !isfinite(dkk)) {
      if (tid == 0) *fail = 1;
      return;
    }
    const double rkk = sqrt(dkk);
    rmax = fmax(rmax, rkk);
    rmin = fmin(rmin, rkk);
    const double inv = 1.0 / dkk;
    for (int j = k + 1 + wave_id(); j < mu; j += 8) {
      const double f = R[k + j * mu] * inv;
      for (int i = k + 1 + (tid & 63); i <= j; i += 64) R[i + j * mu] -= R[k + i * mu] * f;
    }
    if (k >= 1) {
      const double rp = sqrt(dprev);
      for (int j = k - 1 + tid; j < mu; j += 512) R[k - 1 + j * mu] /= rp;
    }
    dprev = dkk;
    __syncthreads();
  }
  if (tid == 0) R[mu - 1 + (mu - 1) * mu] = sqrt(dprev);
  __syncthreads();
  if (!(rmax <= GR_MAXRATIO * rmin)) {
    if (tid == 0) *fail = 1;
    return;
  }
  __shared__ double ez[GR_MAXC];
  __shared__ double kap;
  if (tid < 64) {
    const double k1 = wave_kappa1_upper(mu, (const double*)R, mu, y, ez);
    if (tid == 0) kap = k1;
  }
  __syncthreads();
  if (!(kap <= maxcond)) {
    if (tid == 0) *fail = 1;
    return;
  }
  if (tid < 64) {
    upper_t_solve_any(mu, (const double*)R, mu, rhs, y);   // R^T w = G~[:m, m]
    upper_solve_any(mu, (const double*)R, mu, y, y);       // R y = w
  }
  __syncthreads();
  double* yout = ws + g.oVec + 2 * (long long)m;
  for (int j = tid; j < mu; j += 512) yout[j] = y[j];
  const double* H = d.H;
  const double hlast = H[(long long)(mu - 1) * m1 + mu];
  double* Hh = ws + g.oH;
  for (int x = tid; x < mu * mu; x += 512) {
    const int r = x % mu, c = x / mu;
    double val = H[(long long)c * m1 + r];
    if (c == mu - 1) val += hlast * y[r];
    Hh[x] = val;
  }
}

namespace {
template <typename T>
void pass_launch_t(const SolveDev& d, const LsqrDev& L, hipStream_t st, int first, size_t lds) {
  if (d.nrhs == 1) hipLaunchKernelGGL((k_lsqr_pass<T, true>), dim3(L.nblk), dim3(256), lds, st, d, L, first);
  else hipLaunchKernelGGL((k_lsqr_pass<T, false>), dim3(L.nblk), dim3(256), lds, st, d, L, first);
}
void step_launch(const SolveDev& d, const DenseDev& g, const LsqrDev& L, hipStream_t st, int first) {
  hipLaunchKernelGGL(k_lsqr_step, dim3(d.nrhs), dim3(256), 0, st, d, g, L, first);
}
void lsqr_pass_launch(const SolveDev& d, const LsqrDev& L, int esize, hipStream_t st, int first) {
  const int ch = lsqr_pass1_chunk(d.m, d.nrhs, esize);
  if (ch) {
    const size_t lds = lsqr_pass1_lds(d.m, ch, esize);
    if (esize == 4) {
      if (ch == 128) hipLaunchKernelGGL((k_lsqr_pass1<float, 128>), dim3(L.nblk), dim3(256), lds, st, d, L, first);
      else hipLaunchKernelGGL((k_lsqr_pass1<float, 64>), dim3(L.nblk), dim3(256), lds, st, d, L, first);
    } else {
      if (ch == 128) hipLaunchKernelGGL((k_lsqr_pass1<double, 128>), dim3(L.nblk), dim3(256), lds, st, d, L, first);
      else hipLaunchKernelGGL((k_lsqr_pass1<double, 64>), dim3(L.nblk), dim3(256), lds, st, d, L, first);
    }
    return;
  }
  const size_t lds = lsqr_pass_lds(d.m, d.nrhs);
  if (esize == 4) pass_launch_t<float>(d, L, st, first, lds);
  else pass_launch_t<double>(d, L, st, first, lds);
}
}  // namespace

// Initialisation (u = v_{m+1}, first bidiagonalisation step).
hipError_t lsqr_begin(const SolveDev& d, const DenseDev& g, const LsqrDev& L, int esize, hipStream_t st) {
  const dim3 rg(d.nrhs, (d.m + 3) / 4);
  if (d.m <= 128) hipLaunchKernelGGL(k_lsqr_rinv<2>, rg, dim3(256), 0, st, d, g, L);
  else if (d.m <= 256) hipLaunchKernelGGL(k_lsqr_rinv<4>, rg, dim3(256), 0, st, d, g, L);
  else hipLaunchKernelGGL(k_lsqr_rinv<8>, rg, dim3(256), 0, st, d, g, L);
  lsqr_pass_launch(d, L, esize, st, 1);
  step_launch(d, g, L, st, 1);
  if (d.nrhs > 1) hipLaunchKernelGGL(k_lsqr_alldone, dim3(1), dim3(64), 0, st, d, L);
  return hipGetLastError();
}

// `count` further iterations; launches after every right-hand side stopped return at once.
hipError_t lsqr_iterate(const SolveDev& d, const DenseDev& g, const LsqrDev& L, int esize, hipStream_t st,
                        int count) {
  for (int it = 0; it < count; ++it) {
    lsqr_pass_launch(d, L, esize, st, 0);
    step_launch(d, g, L, st, 0);
    if (d.nrhs > 1) hipLaunchKernelGGL(k_lsqr_alldone, dim3(1), dim3(64), 0, st, d, L);
  }
  return hipGetLastError();
}

hipError_t lsqr_end(const SolveDev& d, const DenseDev& g, const LsqrDev& L, hipStream_t st) {
  hipLaunchKernelGGL(k_lsqr_finish, dim3(d.nrhs), dim3(256), 0, st, d, g, L);
  return hipGetLastError();
}

// The whole refinement as one fixed-length launch sequence (L.maxit iterations).
hipError_t lsqr_launch(const SolveDev& d, const DenseDev& g, const LsqrDev& L, int esize, hipStream_t st) {
  hipError_t e = lsqr_begin(d, g, L, esize, st);
  if (e == hipSuccess) e = lsqr_iterate(d, g, L, esize, st, L.maxit);
  if (e == hipSuccess) e = lsqr_end(d, g, L, st);
  return e;
}

bool gram_ls_supported(const SolveDev& d) { return d.nrhs == 1 && d.m + 1 <= GR_MAXC; }
size_t gram_ls_partial_doubles() { return (size_t)GR_BLOCKS * GR_NT * 256; }

// The exact least-squares solve from the Gram matrix (one right-hand side).
hipError_t gram_ls_launch(const SolveDev& d, const DenseDev& g, double* part, int* fail, int esize, double tol,
                          hipStream_t st) {
  if (!gram_ls_supported(d)) return hipErrorInvalidValue;
  const double maxcond = fmin(GR_MAXCOND, sqrt(fmax(tol, 0.0) / (10.0 * ldexp(1.0, -53))));
  if (esize == 4) hipLaunchKernelGGL(k_vgram<float>, dim3(GR_BLOCKS), dim3(256), 0, st, d, part);
  else hipLaunchKernelGGL(k_vgram<double>, dim3(GR_BLOCKS), dim3(256), 0, st, d, part);
  hipLaunchKernelGGL(k_vgram_reduce, dim3(GR_NT), dim3(256), 0, st, d, g, (const double*)part, GR_BLOCKS);
  hipLaunchKernelGGL(k_vgram_solve, dim3(1), dim3(512), (size_t)d.m * d.m * 8, st, d, g, fail, maxcond);
  return hipGetLastError();
}

hipError_t lsqr_set_attributes() {
  hipError_t e = hipSuccess, r;
  const void* passes[4] = {(const void*)k_lsqr_pass<float, true>, (const void*)k_lsqr_pass<float, false>,
                           (const void*)k_lsqr_pass<double, true>, (const void*)k_lsqr_pass<double, false>};
  const void* passes1[4] = {(const void*)k_lsqr_pass1<float, 128>, (const void*)k_lsqr_pass1<float, 64>,
                            (const void*)k_lsqr_pass1<double, 128>, (const void*)k_lsqr_pass1<double, 64>};
  for (const void* k : passes1)
    if ((r = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 80 * 1024)) != hipSuccess) e = r;
  for (const void* k : passes)
    if ((r = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 120 * 1024)) != hipSuccess) e = r;
  if ((r = hipFuncSetAttribute((const void*)k_vgram_solve, hipFuncAttributeMaxDynamicSharedMemorySize,
                               GR_MAXC * GR_MAXC * 8)) != hipSuccess) e = r;
  return e;
}

}  // namespace fab
