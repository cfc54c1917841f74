// Device-side descriptors and helpers shared by the libfab kernels.
//
// Data layout in HBM for one solve with nrhs right-hand sides:
//   V      basis, (m+1) vectors of n*nrhs elements (FP32 or FP64), vector j at
//          V + j*ldv, element (row r, rhs q) at r*nrhs + q.  Vectors are stored
//          unnormalised: v_j = u_j / eta_j (lazy normalisation).
//   wbuf   CSR only: w~ = A u_{i-1} in FP64, [n][nrhs].
//   H      per rhs, (m+1) x m column-major (ld m+1): the Hessenberg matrix of
//          the Arnoldi-like decomposition, eq. (3) of the paper.
//   S      per rhs, s x (m+1) column-major (ld s): Theta u_j (unnormalised).
//   part / npart / skpart: per-block partial sums, reduced in a fixed order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fab {

constexpr int KMAX = 8;          // largest truncation window k
constexpr int ZMAX = 16;         // largest sparse-sign zeta
constexpr int NSLOT = KMAX + 1;  // dot slots per rhs: k window dots + ||w||^2
constexpr int BLOCK = 256;       // threads per streaming block
constexpr int TILE_ELEMS = 4096; // max elements (rows * nrhs) per tile

// Column pointers of a block of single-rhs requests (at most 32).
struct ColPtrs { const double* p[32]; };
struct OutPtrs { double* p[32]; };

// Operator path of the streaming kernels: OP_STENCIL recomputes A u inside
// the passes; OP_CSR reads w~ = A u from wbuf, written by a product launch
// before the passes (a CSR matrix, or A applied twice for the sign function).
enum OpKind { OP_STENCIL = 0, OP_CSR = 1 };
// How that product launch forms w~ (operator_product, k_csr.hip).
enum ProdKind { PROD_FUSED = 0, PROD_CSR = 1, PROD_SQ_STENCIL = 2, PROD_SQ_CSR = 3 };
enum SketchKind { SK_SRHT = 1, SK_SPARSE = 2 };

struct SolveDev {
  // problem shape
  int n;                 // rows
  int nrhs, lognrhs;     // rhs count (power of two <= 32)
  int m, k, s, zeta;
  // operator
  int op;                // OpKind of the streaming kernels
  int prod;              // ProdKind: how w~ is formed for op == OP_CSR
  int nx, ny, nz;
  double c[7];           // stencil coefficients (centre, x-, x+, y-, y+, z-, z+)
  const int* rowptr;
  const int* col;
  const float* val;
  // basis
  void* V;
  long long ldv;         // n * nrhs
  double* wbuf;          // OP_CSR: w~ [n][nrhs]
  double* wtmp;          // PROD_SQ_*: A u, the intermediate of A (A u) [n][nrhs]
  const double* b;       // right-hand sides [n][nrhs]
  // small state, per rhs
  double* H;             // [nrhs][(m+1)*m]
  double* eta;           // [nrhs][m+1]
  double* wnorm;         // [nrhs][m+1]
  double* coef;          // [nrhs][NSLOT]
  double* S;             // [nrhs][s*(m+1)]
  // partition and partials
  int log_tile;          // tile = 2^log_tile elements (9 or 12)
  int rows_per_tile, log_rows;   // R = rows per tile = 2^log_tile / nrhs
  int ntiles;            // ceil(n / R)
  int nblk;              // streaming blocks (tiles are strided over blocks)
  int nred;              // sketch-reduction blocks (leading blocks of the update kernel)
  double* part;          // [nblk][nrhs][NSLOT]
  double* npart;         // [nblk][nrhs]
  double* skpart;        // two buffers [2][s*nrhs][nblk]: column c uses buffer c & 1
  long long skstride;    // s*nrhs*nblk
  unsigned* counter;     // last-block ticket
  int* status;           // [0] m_used, [1] breakdown, [2] non-finite
  // sketch
  int sketch;            // SketchKind
  int sk_slices;         // sparse sign: LDS accumulators per block (1, or one per wave)
  int sk_reg;            // SRHT: 1 = each thread holds its sketch accumulators in registers
  int tgroups;           // streaming blocks form tgroups groups (blk mod tgroups), 8 or 1
  long long tchunk;      // tiles per group: group g walks tiles [g*tchunk, (g+1)*tchunk)
  int wtp, wc, wpen;     // pencil walk (wtp > 0): tiles per z-plane, tiles per pencil row,
                         // pencils per group (3D stencils with large planes)
  int wz;                // z-march walk (> 0: tiles per block; wtp tiles per plane, wc
                         // tile columns per group)
  const int* srht_rows;  // [s] sampled rows of the padded Hadamard transform
  unsigned long long key_a, key_b;   // SRHT: signs key; sparse: rows key, signs key
  double sk_scale;       // 1/sqrt(s) (SRHT) or 1/sqrt(zeta) (sparse sign)
  double unit_round;     // unit roundoff of the basis storage
};

// Window length a streaming kernel is instantiated for (k <= KT).
__host__ __device__ constexpr int window_kt(int k) { return k <= 2 ? 2 : (k <= 4 ? 4 : 8); }
// SRHT with 8 rhs: sampled rows (multiples of the block size) whose sums a
// thread of k_update keeps in registers, by window length: what fits beside
// the rest in 256 VGPRs (2 waves per SIMD).  0: every sum in LDS and one tile
// buffer.  The host sizes k_update's LDS from the same function.
__host__ __device__ constexpr int srht_qrows(int kt) { return kt <= 2 ? 1 : (kt <= 4 ? 2 : 0); }

// Per-rhs workspace of the small dense stages (FP64, column-major).
constexpr int MAXCOEF = 64;
constexpr int NINFO = 20;
struct DenseDev {
  int m, s, nrhs;
  long long stride;      // doubles per rhs
  double* base;
  // per-rhs regions: Householder workspace [s*(m+1)], R [m*m], compressed
  // matrices [3][m*m] (one per variant), scratch [9*m*m], vectors [8(m+1)+32], info
  long long oW, oR, oH, oM, oVec, oInfo;
  int ls_mode;           // 1 sketch-and-solve, 2 none
  int fkind;             // 1 exp, 2 pow, 3 poly
  int nvar;              // f evaluations per rhs: 1, or 3 with the a-posteriori estimates
  double alpha, sigma, p;
  double unit_round;     // unit roundoff of the basis storage (rounding estimate)
  int ncoef;
  double coef[MAXCOEF];
};

// Per-rhs info block (NINFO doubles), copied to the host after every solve.
enum {
  INFO_KAPPA = 0,    // kappa(R) of the sketched basis (|r_jj| max / min)
  INFO_HLAST = 1,    // h_{m+1,m}
  INFO_BETA = 2,     // ||b||
  INFO_FAIL = 3,     // 1: singular / non-finite small problem, 2: Schur iteration failed
  INFO_NSQ = 4,      // exp: scaling steps
  INFO_SCHUR_IT = 5, // pow: Schur sweeps; exp: Taylor degree
  INFO_NRM = 6,      // exp: ||alpha H_hat||_1
  INFO_LSQR_IT = 7,  // LSQR refinement iterations
  INFO_MD = 8,       // order m_used - d of the convergence-check variant
  INFO_GATE = 9,     // ||R (c_y - c_0)|| / ||R c_y||
  INFO_ROUND = 10,   // u sum_j |c_j| ||R e_j|| / ||R c||
  INFO_CONV = 11,    // ||R (c - [c_{m-d}; 0])|| / ||R c||
  INFO_VFAIL = 12,   // [12 + v]: failure of variant v's f evaluation
  INFO_LSQR_RATIO = 15,  // Paige-Saunders measure ||M^T r|| / (||M||_F ||r||) of the last LSQR iteration
  INFO_LSQR_LIMIT = 16   // 1: LSQR stopped at its iteration limit before meeting its test
};

// LSQR refinement state (see k_lsqr.hip)
struct LsqrDev {
  double* u;             // [n][nrhs] FP64 LSQR vector (unnormalised)
  double* part;          // [nblk][nrhs][m+1] per-block dots and norm
  double* st;            // [nrhs][stride] per-rhs vectors and scalars
  long long stride;
  int* alldone;          // every rhs stopped: remaining launches return
  double* rinv;          // [nrhs][2][m*m]: X = R_m^{-1} (upper, ld m_used) and X^T
  int nblk, maxit;
  double tol;            // stop when ||M^T r|| <= tol ||M||_F ||r|| (Paige-Saunders)
};

// The f evaluations of the dense tail.  Variant 0 is the result (H_hat of
// order m_used); with the estimates, variant 1 is H_m without the
// least-squares correction (the cheaper approximation, eq. (8)) and variant 2
// the compression at order m_used - d.  Each has its matrix (ld = its order),
// output vector and scratch.
struct DenseVariant {
  int dim;
  const double* H;
  double* c;
  double* scratch;      // 3 m*m doubles
  double* info;
};
__device__ inline DenseVariant dense_variant(const SolveDev& d, const DenseDev& g, int q, int v) {
  double* ws = g.base + (long long)q * g.stride;
  const long long mm = (long long)g.m * g.m;
  DenseVariant r;
  const int mu = d.status[4 + 2 * q];
  r.dim = v == 2 ? (int)ws[g.oInfo + INFO_MD] : mu;
  r.H = ws + g.oH + v * mm;
  r.c = ws + g.oVec + (v == 0 ? 0 : (v == 1 ? 5 : 6) * (long long)(g.m + 1));
  r.scratch = ws + g.oM + 3 * v * mm;
  r.info = ws + g.oInfo;
  return r;
}

// ---------------------------------------------------------------- wave helpers
// Index of this thread's wave in the workgroup, marked wave-uniform so that
// branches on it stay scalar.
__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Value of a double in lane `lane` (wave-uniform index) of this wave.
__device__ inline double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Back substitution U x = z for upper-triangular U (order n <= 64 R,
// column-major, leading dimension ldu) by one wave: rows lane + 64 u stay in
// registers and x_j is read from its owner lane, so no barrier is needed.  A
// zero diagonal entry gives x_j = 0.  z and x may alias.
template <int R>
__device__ void wave_upper_solve(int n, const double* U, long long ldu, const double* z, double* x) {
  const int lane = threadIdx.x & 63;
  double y[R];
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int r = lane + 64 * u;
    y[u] = r < n ? z[r] : 0.0;
  }
  for (int j = n - 1; j >= 0; --j) {
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
      else if (r < j) y[u] -= U[r + (long long)j * ldu] * xj;
    }
  }
#pragma unroll
  for (int u = 0; u < R; ++u) {
    const int r = lane + 64 * u;
    if (r < n) x[r] = y[u];
  }
}

// ---------------------------------------------------------------- SplitMix64
// Counter-based SplitMix64 (Steele, Lea & Flood 2014): out(key, i) is the
// i-th output of the generator whose state starts at `key`; stream keys are
// outputs of the generator seeded with the user seed.
constexpr unsigned long long GOLDEN_GAMMA = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline unsigned long long sm64_finalise(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ inline unsigned long long sm64_out(unsigned long long key, unsigned long long i) {
  return sm64_finalise(key + (i + 1ull) * GOLDEN_GAMMA);
}

// Sparse-sign pattern of column `r` of Theta: zeta distinct rows in [0, s)
// (Floyd's sampling) and a sign bit word.
__device__ inline void sparse_sign_column(unsigned long long key_rows, unsigned long long key_signs,
                                          int r, int s, int zeta, int* rows, unsigned long long* sbits) {
  const unsigned half = (unsigned)(zeta + 1) >> 1;
  unsigned long long w = 0;
#pragma unroll
  for (int t = 0; t < ZMAX; ++t) {
    if (t < zeta) {
      if ((t & 1) == 0) w = sm64_out(key_rows, (unsigned long long)r * half + (unsigned)(t >> 1));
      unsigned h = (t & 1) ? (unsigned)(w & 0xFFFFFFFFull) : (unsigned)(w >> 32);
      unsigned j = (unsigned)(s - zeta + t);
      unsigned q = (unsigned)(((unsigned long long)h * (unsigned long long)(j + 1u)) >> 32);
      bool taken = false;
#pragma unroll
      for (int u = 0; u < ZMAX; ++u)
        if (u < t && rows[u] == (int)q) taken = true;
      rows[t] = taken ? (int)j : (int)q;
    }
  }
  *sbits = sm64_out(key_signs, (unsigned long long)r);
}

// ---------------------------------------------------------------- reductions
// Sum over the lanes of a wave that share the same rhs (lane & (nrhs-1)).
// Fixed xor-butterfly order: deterministic.
__device__ inline double wave_sum_rhs(double v, int nrhs) {
  for (int off = 32; off >= nrhs; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Tiles of streaming block blk: blocks blk = g + tgroups * c form group g.
// Consecutive workgroups of a launch are dispatched round-robin over the 8
// XCDs, so with tgroups = 8 one group runs on one XCD.  The block visits
// tiles walk_tile(w, u) for u = u0, u0 + step, ... < uhi (the members of a
// group interleaved), so that neighbouring tiles -- the stencil's y and z
// neighbours -- are read through that XCD's L2 while still resident:
//  * linear walk: group g takes the contiguous tiles [g tchunk, (g+1) tchunk);
//  * pencil walk (3D stencil whose z-plane is large): a z-plane of wtp tiles
//    is cut into pencils of wc consecutive tiles; group g takes pencils
//    g, g + 8, ... (wpen of them) and walks each through all z-planes, so
//    the planes z - 1, z, z + 1 of a pencil are touched close together;
//  * z-march (the same case, when each group can own whole tile columns):
//    tile (z, y) = z wtp + y; group g owns the wc columns y in
//    [g wc, (g+1) wc) through all planes, ordered column by column with z
//    fastest, and block u of the group walks its own wz consecutive tiles
//    of that order (u0 = u wz, step 1).  A block's next tile is the
//    z + 1 neighbour of its current one (its z - 1 neighbour is the tile it
//    did before), and the group's blocks advance through the planes side by
//    side, so a tile's y-neighbours are read by sibling blocks of the same
//    XCD at the same time.
struct TileWalk {
  int u0, uhi, step, g;
  long long lo;
};
__device__ inline TileWalk tile_walk(const SolveDev& d, int blk) {
  const int G = d.tgroups;
  TileWalk w;
  w.g = blk % G;
  w.u0 = blk / G;
  w.step = d.nblk / G;
  if (d.wz > 0) {
    w.lo = 0;
    w.u0 = (blk / G) * d.wz;
    const int tot = d.wc * d.nz;
    w.uhi = w.u0 + d.wz < tot ? w.u0 + d.wz : tot;
    w.step = 1;
  } else if (d.wtp > 0) {
    w.lo = 0;
    w.uhi = d.wpen * d.nz * d.wc;
  } else {
    w.lo = (long long)w.g * d.tchunk;
    const long long h = w.lo + d.tchunk < (long long)d.ntiles ? w.lo + d.tchunk : (long long)d.ntiles;
    w.uhi = (int)(h - w.lo);
  }
  return w;
}
__device__ inline int walk_tile(const SolveDev& d, const TileWalk& w, int u) {
  if (d.wz > 0) {
    const int col = u / d.nz, z = u - col * d.nz;
    return z * d.wtp + w.g * d.wc + col;
  }
  if (d.wtp <= 0) return (int)(w.lo + u);
  const int zc = d.nz * d.wc;
  const int j = u / zc, rem = u - j * zc;
  const int z = rem / d.wc, cc = rem - z * d.wc;
  return z * d.wtp + (w.g + 8 * j) * d.wc + cc;
}

}  // namespace fab
