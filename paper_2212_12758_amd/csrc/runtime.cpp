// libfab host runtime: the C ABI of include/fab.h.
//
//  * Arena: one device allocation (caller-provided or owned) carved by a
//    first-fit allocator with coalescing; matrices and per-request
//    workspaces live in it, so admission control is "does the workspace fit".
//  * Solve plan: sizes, partition of the rows into tiles, device descriptors.
//  * Launch sequence per solve (all on one stream, no host round trip):
//      init -> start (u_0 = b) -> m x (dots, update) -> finish -> dense tail
//      (sketched QR / least squares, f(H_hat) e_1, weights) -> combine.
//  * Serving loop: fab_submit queues a request; a scheduler thread admits
//    queued requests in FIFO order whenever their workspace fits next to the
//    running ones, runs each admitted request on its own stream (so work of
//    different requests overlaps on the device), and retires them as their
//    completion events fire.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/fab.h"
#include "fab_dev.h"

namespace fab {
hipError_t basis_set_attributes();
hipError_t basis_start(const SolveDev& d, int esize, hipStream_t st, size_t lds);
hipError_t basis_dots(const SolveDev& d, int esize, int i, hipStream_t st);
hipError_t basis_update(const SolveDev& d, int esize, int i, hipStream_t st, size_t lds);
hipError_t basis_finish(const SolveDev& d, int esize, hipStream_t st);
hipError_t basis_combine(const SolveDev& d, int esize, const double* cf, int mmax, double* out, hipStream_t st);
hipError_t dense_tail(const SolveDev& d, const DenseDev& g, double* cf, double* fq, hipStream_t st);
size_t fsqrt_partials_doubles(int m, int nrhs);
hipError_t fsqrt_set_attributes();
hipError_t zero_fill(void* p, size_t bytes, hipStream_t st);
hipError_t srht_sample_rows(int* rows, long long npad, int s, unsigned long long key, hipStream_t st);
hipError_t dense_set_attributes();
hipError_t dense_after_refine(const SolveDev& d, const DenseDev& g, double* cf, double* fq, hipStream_t st);
hipError_t lsqr_launch(const SolveDev& d, const DenseDev& g, const LsqrDev& L, int esize, hipStream_t st);
hipError_t lsqr_begin(const SolveDev& d, const DenseDev& g, const LsqrDev& L, int esize, hipStream_t st);
hipError_t lsqr_iterate(const SolveDev& d, const DenseDev& g, const LsqrDev& L, int esize, hipStream_t st,
                        int count);
hipError_t lsqr_end(const SolveDev& d, const DenseDev& g, const LsqrDev& L, hipStream_t st);
bool gram_ls_supported(const SolveDev& d);
size_t gram_ls_partial_doubles();
hipError_t gram_ls_launch(const SolveDev& d, const DenseDev& g, double* part, int* fail, int esize, double tol,
                          hipStream_t st);
hipError_t lsqr_set_attributes();
hipError_t bg_apply(const SolveDev& d, int esize, int i, hipStream_t st, size_t lds);
hipError_t bg_reduce(const SolveDev& d, int col, hipStream_t st);
hipError_t bg_gs(const SolveDev& d, double* cf, int i, int passes, hipStream_t st);
hipError_t bg_update(const SolveDev& d, int esize, const double* cf, int i, hipStream_t st);
hipError_t bg_set_attributes();
hipError_t apply_operator(const SolveDev& d, const double* x, double* y, hipStream_t st);
hipError_t wh_col(const SolveDev& d, const DenseDev& g, int a, int check, double thresh, int* flag,
                  hipStream_t st);
hipError_t wh_whiten(const SolveDev& d, const DenseDev& g, int esize, int i, hipStream_t st);
hipError_t wh_set_attributes();

// Whitening (FAB_BASIS_WHITENED): test the sketch condition every WH_EVERY
// steps against WH_THRESH (the threshold of Section 5.1.3).
constexpr int WH_EVERY = 5;
constexpr double WH_THRESH = 1000.0;
// Internal status of enqueue_solve (never returned through the C ABI): an
// FP32 attempt under FAB_PREC_AUTO stopped at its whitening trigger, since
// its result could not be accepted (the caller recomputes with FP64).
constexpr int RC_RERUN_FP64 = 100;
size_t lsqr_state_stride(int m);
size_t lsqr_pass_lds(int m, int nrhs);
int lsqr_pass1_chunk(int m, int nrhs, int esize);
hipError_t gather_cols(const ColPtrs& src, int logg, long long n, double* dst, hipStream_t st);
hipError_t scatter_cols(const double* src, int logg, long long n, const OutPtrs& dst, hipStream_t st);
// Per-device address of the static scratch of fab_solve_noalloc (noalloc.hip).
int noalloc_setup(int device);
}  // namespace fab

using namespace fab;

// ============================================================== arena allocator
namespace {

struct Arena {
  char* base = nullptr;
  size_t size = 0;
  bool owned = false;
  std::map<size_t, size_t> free_;   // offset -> length
  size_t in_use = 0;

  void init(char* b, size_t n) {
    base = b;
    size = n;
    free_.clear();
    free_[0] = n;
    in_use = 0;
  }
  // first fit, 256-byte aligned lengths; returns nullptr if no block fits
  void* alloc(size_t n) {
    n = (n + 255) & ~size_t(255);
    if (n == 0) n = 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        const size_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > n) free_[off + n] = len - n;
        in_use += n;
        sizes_[off] = n;
        return base + off;
      }
    }
    return nullptr;
  }
  // Long-lived regions (resident matrices, cached sketch rows) are carved from
  // the top of the highest free block that fits, so that they never split the
  // space left for the large per-request workspaces, which come from the bottom.
  void* alloc_high(size_t n) {
    n = (n + 255) & ~size_t(255);
    if (n == 0) n = 256;
    for (auto it = free_.rbegin(); it != free_.rend(); ++it) {
      if (it->second >= n) {
        const size_t off = it->first + it->second - n;
        if (it->second == n) free_.erase(std::next(it).base());
        else it->second -= n;
        in_use += n;
        sizes_[off] = n;
        return base + off;
      }
    }
    return nullptr;
  }
  void release(void* p) {
    if (!p) return;
    const size_t off = (char*)p - base;
    auto sit = sizes_.find(off);
    if (sit == sizes_.end()) return;
    size_t n = sit->second;
    sizes_.erase(sit);
    in_use -= n;
    size_t o = off;
    auto nx = free_.lower_bound(o);
    if (nx != free_.end() && nx->first == o + n) {
      n += nx->second;
      free_.erase(nx);
    }
    auto pv = free_.lower_bound(o);
    if (pv != free_.begin()) {
      --pv;
      if (pv->first + pv->second == o) {
        o = pv->first;
        n += pv->second;
        free_.erase(pv);
      }
    }
    free_[o] = n;
  }
  bool could_ever_fit(size_t n) const { return ((n + 255) & ~size_t(255)) <= size; }

 private:
  std::map<size_t, size_t> sizes_;
};

double now_us() {
  using namespace std::chrono;
  return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct fab_matrix_s {
  fab_ctx ctx = nullptr;
  int op = OP_STENCIL;
  int dim = 2, nx = 1, ny = 1, nz = 1;
  double c[7] = {0};
  int n = 0;
  long long nnz = 0;
  int* rowptr = nullptr;
  int* col = nullptr;
  float* val = nullptr;
  std::atomic<int> refs{0};
};

namespace {

struct Plan {
  // inputs
  fab_matrix A = nullptr;
  const double* b = nullptr;
  double* out = nullptr;
  int nrhs = 1;
  fab_func f{};
  std::vector<double> coef;
  fab_params p{};
  int esize = 4;
  int nvar = 1;                // dense f evaluations per rhs (3 with the a-posteriori estimates)
  bool lsqr = false;           // workspace for the LSQR refinement is planned
  bool bg = false;             // basis by Gram-Schmidt on the sketch (Algorithm 1)
  bool whiten = false;         // truncated basis, whitened on a condition trigger, then Algorithm 1
  int whitened_at = 0;         // step at which the last solve whitened (0: never)
  size_t oBgCf = 0;            // Algorithm 1 update weights [nrhs][m+2]
  size_t oFq = 0;              // quadrature partial sums of the square root (FAB_F_POW)
  bool sign = false;           // FAB_F_SIGN: the basis is built for A^2 (A applied twice) from A b
  fab_func forig{};            // the caller's f (kind FAB_F_SIGN)
  size_t oSignB = 0;           // A b, FP64 [n][nrhs]
  size_t oWtmp = 0;            // A u, the intermediate of A (A u), FP64 [n][nrhs]
  bool gram = false;           // FAB_LS_GRAM with one rhs and m + 1 <= 128: exact least squares
  bool gram_used = false;      // the last refinement solved through the Gram matrix
  size_t oGpart = 0, oGflag = 0;
  size_t oWflag = 0;           // whitening trigger flag
  int lnblk = 0;               // LSQR pass blocks
  size_t oLu = 0, oLpart = 0, oLst = 0, oLflag = 0, oLri = 0;
  // derived
  int LT = 12, R = 0, logR = 0, ntiles = 0, nblk = 0, nred = 0;
  long long ldv = 0;
  size_t lds_update = 0;
  size_t lds_kupdate = 0;      // dynamic LDS of k_update (smaller with register SRHT accumulators)
  int sk_slices = 1;
  int sk_reg = 0;              // SRHT accumulators in registers (k_update)
  int tgroups = 1;             // XCD groups of the streaming blocks
  int wtp = 0, wc = 0, wpen = 0;   // pencil walk of the streaming blocks (wtp = 0: linear)
  int wz = 0;                      // z-march walk: tiles per block (0: not used)
  size_t bytes = 0;
  // offsets in the workspace
  size_t oV, oW, oH, oEta, oWn, oCoef, oS, oPart, oNpart, oSk, oCnt, oStatus, oRows, oDense, oCf, oInfoHost;
  size_t dense_stride = 0;  // doubles per rhs
  size_t oDW, oDR, oDH, oDM, oDVec, oDInfo;
};

int ilog2(long long v) {
  int l = 0;
  while ((1LL << l) < v) ++l;
  return l;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int make_plan(fab_matrix A, int nrhs, const fab_func& fin, const fab_params* pp, int esize, Plan& P) {
  if (!A || !pp) return FAB_EINVAL;
  // sign(A) b = (A^2)^{-1/2} (A b): plan the inverse square root with the
  // operator A^2, applied as two products with A in every step
  fab_func f = fin;
  const bool sign = fin.kind == FAB_F_SIGN;
  if (sign) {
    P.forig = fin;
    f = fab_func{FAB_F_POW, 0.0, 0.0, -0.5, nullptr, 0};
  }
  P.sign = sign;
  const fab_params& p = *pp;
  const long long n = A->n;
  if (nrhs < 1 || nrhs > 32 || (nrhs & (nrhs - 1))) return FAB_EINVAL;
  if (p.m < 1 || p.m >= n || p.m > 500) return FAB_EINVAL;
  if (p.basis != FAB_BASIS_TRUNCATED && p.basis != FAB_BASIS_SKETCHED_GS && p.basis != FAB_BASIS_SKETCHED_GS2 &&
      p.basis != FAB_BASIS_WHITENED)
    return FAB_EINVAL;
  const bool whiten = p.basis == FAB_BASIS_WHITENED;
  const bool bg = p.basis == FAB_BASIS_SKETCHED_GS || p.basis == FAB_BASIS_SKETCHED_GS2;
  if (p.ls_maxit < 0 || p.ls_maxit > 1024) return FAB_EINVAL;
  if (!bg && (p.k < 1 || p.k > KMAX)) return FAB_EINVAL;
  if (p.sketch != FAB_SKETCH_SRHT && p.sketch != FAB_SKETCH_SPARSE_SIGN) return FAB_EINVAL;
  const long long npad = 1LL << ilog2(n);
  if (p.s <= p.m || p.s > 8192 || p.s > npad) return FAB_EINVAL;
  if (p.sketch == FAB_SKETCH_SPARSE_SIGN && (p.zeta < 1 || p.zeta > ZMAX || p.zeta > p.s)) return FAB_EINVAL;
  if (p.ls_mode < FAB_LS_AUTO || p.ls_mode > FAB_LS_GRAM) return FAB_EINVAL;
  if (f.kind == FAB_F_POW) {
    if (!(f.p == 0.5 || f.p == -0.5)) return FAB_EINVAL;
  } else if (f.kind == FAB_F_POLY) {
    if (f.ncoef < 1 || f.ncoef > MAXCOEF || !f.coef) return FAB_EINVAL;
  } else if (f.kind != FAB_F_EXP) {
    return FAB_EINVAL;
  }
  P.A = A;
  P.nrhs = nrhs;
  P.f = f;
  if (f.kind == FAB_F_POLY) P.coef.assign(f.coef, f.coef + f.ncoef);
  P.p = p;
  if (bg) P.p.k = 1;   // the window is not used
  P.bg = bg;
  P.whiten = whiten;
  P.esize = esize;
  P.nvar = (p.prec == FAB_PREC_AUTO || p.ls_mode == FAB_LS_AUTO) ? 3 : 1;
  // tiles of 2^LT elements (rows x rhs): 2048 for large problems, 512 below
  // 2^20 elements so that smaller problems still spread over many blocks
  const long long nel = n * nrhs;
  P.LT = nel >= (1LL << 20) ? 11 : 9;
  const long long tile = 1LL << P.LT;
  P.R = (int)(tile / nrhs);
  P.logR = ilog2(P.R);
  P.ntiles = (int)((nel + tile - 1) / tile);
  // at most 512 blocks: every block of the update pass first reduces the
  // previous pass's per-block partials (fixed order), a cost that grows with
  // the square of the block count (2048 blocks of 512 elements: 0.37 GB of
  // partial reads per launch at n = 2^20)
  P.nblk = std::min(P.ntiles, 512);
  const long long snr = (long long)p.s * nrhs;
  P.nred = (int)std::max<long long>(1, std::min<long long>((snr + 7) / 8, 128));   // one per 8 sketch rows
  // streaming blocks in 8 XCD groups when the grid divides; the leading
  // sketch-reduction blocks of the update pass are a multiple of 8 then, so a
  // block index means the same XCD in both passes of a step
  P.tgroups = (P.nblk >= 8 && P.nblk % 8 == 0) ? 8 : 1;
  if (P.tgroups == 8) P.nred = (P.nred + 7) & ~7;
  // 3D stencil whose z-plane of one vector exceeds 256 KB: pencils of at most
  // 256 KB per plane walked through z, narrow enough that the members of a
  // group work on at least 4 consecutive planes of their pencil at a time, so
  // a tile's z-neighbours are being read by sibling blocks of the same XCD
  // (a whole plane per vector no longer fits its L2)
  P.wtp = P.wc = P.wpen = P.wz = 0;
  {
    const long long plane = (long long)A->nx * A->ny;   // rows per z-plane
    const long long rows_tile = tile / nrhs;
    const long long tile_bytes = tile * esize;
    const bool big_planes = A->op == OP_STENCIL && !sign && A->nz > 1 && P.tgroups == 8 &&
                            plane % rows_tile == 0 && plane * nrhs * esize > (256LL << 10);
    // z-march when the tiles of a plane split evenly over the 8 groups (each
    // block then reads its tiles' z-neighbours as its previous and next
    // tiles; the pencils below keep 4 planes per group in flight, whose
    // z-neighbours no longer all stay in L2 while the window streams past)
    if (big_planes && (plane / rows_tile) % 8 == 0) {
      const long long tp = plane / rows_tile, cols = tp / 8;
      const long long per_blk = (cols * A->nz + P.nblk / 8 - 1) / (P.nblk / 8);
      P.wtp = (int)tp;
      P.wc = (int)cols;
      P.wz = (int)per_blk;
    } else if (big_planes) {
      const long long tp = plane / rows_tile;
      long long c = tp / 8;
      while (c > 1 && (c * tile_bytes > (256LL << 10) || 4 * c > P.nblk / 8)) c /= 2;
      if (c >= 1 && tp % (8 * c) == 0) {
        P.wtp = (int)tp;
        P.wc = (int)c;
        P.wpen = (int)(tp / (8 * c));
      }
    }
  }
  P.lds_update = (size_t)(snr + (p.sketch == FAB_SKETCH_SRHT ? tile + tile / 32 : 0)) * 8 + (size_t)p.s * 4;
  if (P.lds_update > 160 * 1024) return FAB_EINVAL;
  // sparse sign with 4-wave blocks: one LDS accumulator per wave when the four
  // fit in 96 KB, which makes the sketch sums independent of wave timing
  P.sk_slices = 1;
  if (p.sketch == FAB_SKETCH_SPARSE_SIGN && P.LT == 11 && (size_t)snr * 4 * 8 <= 96 * 1024) {
    P.sk_slices = 4;
    P.lds_update = (size_t)snr * 4 * 8 + (size_t)p.s * 4;
  }
  // SRHT with one rhs: each thread of k_update holds its s/BLOCK sketch
  // accumulators in registers when there are at most 4
  P.lds_kupdate = P.lds_update;
  P.sk_reg = 0;
  if (p.sketch == FAB_SKETCH_SRHT && nrhs == 1 && snr <= 4LL * (tile / 8)) {
    P.sk_reg = 1;
    P.lds_kupdate = (size_t)(tile + tile / 32) * 8 + (size_t)p.s * 4;
  }
  // SRHT with 8 rhs: the sums of the first srht_qrows(KT) * BLOCK sampled
  // rows in registers, two tile buffers (as k_update, KT the window length
  // it is instantiated for); never more than lds_update
  const int kt = window_kt(P.p.k);
  if (p.sketch == FAB_SKETCH_SRHT && nrhs == 8 && srht_qrows(kt) > 0) {
    const long long rreg = (long long)srht_qrows(kt) * (tile / 8);
    const long long sacc = p.s > rreg ? p.s - rreg : 0;
    P.lds_kupdate = (size_t)(2 * (tile + tile / 32) + sacc * nrhs) * 8 + (size_t)p.s * 4;
  }
  P.ldv = (nel + 63) & ~63LL;
  const int m = p.m, s = p.s;
  // dense workspace per rhs
  size_t o = 0;
  P.oDW = o; o += (size_t)s * (m + 1);
  P.oDR = o; o += (size_t)(m + 1) * (m + 1);
  P.oDH = o; o += (size_t)3 * m * m;     // one compressed matrix per variant
  P.oDM = o; o += (size_t)9 * m * m;     // 3 m*m scratch per variant
  P.oDVec = o; o += (size_t)8 * (m + 1) + 32;   // vectors c, y, ...; exp parameter block behind them
  P.oDInfo = o; o += NINFO;
  P.dense_stride = (o + 31) & ~size_t(31);
  // workspace layout
  size_t w = 0;
  auto take = [&](size_t bytes) { size_t at = w; w = align256(w + bytes); return at; };
  P.oV = take((size_t)(m + 1) * P.ldv * esize);
  P.oW = (A->op == OP_CSR || sign) ? take((size_t)n * nrhs * 8) : 0;
  P.oWtmp = sign ? take((size_t)n * nrhs * 8) : 0;
  P.oH = take((size_t)nrhs * (m + 1) * m * 8);
  P.oEta = take((size_t)nrhs * (m + 1) * 8);
  P.oWn = take((size_t)nrhs * (m + 1) * 8);
  P.oCoef = take((size_t)nrhs * NSLOT * 8);
  P.oS = take((size_t)nrhs * s * (m + 1) * 8);
  P.oPart = take((size_t)P.nblk * nrhs * NSLOT * 8);
  P.oNpart = take((size_t)2 * P.nblk * nrhs * 8);
  P.oSk = take((size_t)2 * ((snr + 7) & ~7LL) * P.nblk * 8);
  P.oCnt = take(256);
  P.oStatus = take((size_t)(4 + 2 * nrhs) * 4);
  P.oRows = take(256);   // unused: sampled SRHT rows live in the context's cache
  P.oDense = take(P.dense_stride * nrhs * 8);
  P.oCf = take((size_t)nrhs * (m + 1) * 8);
  if (bg || whiten) P.oBgCf = take((size_t)nrhs * (m + 2) * 8);
  if (whiten) P.oWflag = take(256);
  if (f.kind == FAB_F_POW) P.oFq = take(fsqrt_partials_doubles(m, nrhs) * 8);
  if (sign) P.oSignB = take((size_t)n * nrhs * 8);
  // LSQR refinement (FAB_LS_AUTO when the gate fails, FAB_LS_LSQR always)
  if (p.ls_mode == FAB_LS_AUTO || p.ls_mode == FAB_LS_LSQR || p.ls_mode == FAB_LS_GRAM) {
    const bool fits = lsqr_pass_lds(m, nrhs) <= 120 * 1024;
    // Algorithm 3 needs the refinement: the sketched problem is trivial for
    // a sketch-orthonormal basis
    if (!fits && (p.ls_mode == FAB_LS_LSQR || p.ls_mode == FAB_LS_GRAM || bg || whiten)) return FAB_EINVAL;
    if (fits) {
      P.lsqr = true;
      // the one-read pass (one rhs) loops over chunks of ch elements
      const int ch = lsqr_pass1_chunk(m, nrhs, esize);
      P.lnblk = (int)std::min<long long>((nel + (ch ? ch : 2048) - 1) / (ch ? ch : 2048), 512);
      P.oLu = take((size_t)nel * 8);
      P.oLpart = take((size_t)P.lnblk * nrhs * (m + 1) * 8);
      P.oLst = take((size_t)nrhs * lsqr_state_stride(m) * 8);
      P.oLflag = take(256);
      P.oLri = take((size_t)nrhs * 2 * m * m * 8);   // R_m^{-1} and its transpose
    }
  }
  P.gram = p.ls_mode == FAB_LS_GRAM && nrhs == 1 && m + 1 <= 128;
  if (P.gram) {
    P.oGpart = take(gram_ls_partial_doubles() * 8);
    P.oGflag = take(256);
  }
  P.bytes = w;
  return FAB_OK;
}

struct Request;

// Optional per-launch timing with HIP events on the solve's stream.
struct Prof {
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::pair<int, size_t>> marks;   // (class, index of the start event)
  double total_ms[FAB_K_NCLASS] = {0};
  long long count[FAB_K_NCLASS] = {0};
  int mask = 0;
  hipEvent_t next() {
    if (used == pool.size()) {
      hipEvent_t e;
      hipEventCreate(&e);
      pool.push_back(e);
    }
    return pool[used++];
  }
  void begin(int cls, hipStream_t st) {
    marks.emplace_back(cls, used);
    hipEventRecord(next(), st);
  }
  void end(hipStream_t st) { hipEventRecord(next(), st); }
  void harvest() {   // after the stream was synchronised
    for (auto& mk : marks) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, pool[mk.second], pool[mk.second + 1]) == hipSuccess) {
        total_ms[mk.first] += ms;
        count[mk.first] += 1;
      }
    }
    marks.clear();
    used = 0;
  }
};

}  // namespace

// Fixed-size pinned host slots (a request's info block, a whitening flag),
// allocated in chunks and reused: freeing pinned memory synchronises the
// whole device, which would drain every serving stream each time a request
// completes.  Chunks are freed at fab_finalize only.  Caller holds the
// context's mutex.
struct PinnedSlots {
  static constexpr size_t SLOT = 6144;   // >= host_info_doubles(32) * 8
  static constexpr int PER_CHUNK = 64;
  std::vector<void*> chunks, free_;
  void* get() {
    if (free_.empty()) {
      void* c = nullptr;
      if (hipHostMalloc(&c, SLOT * PER_CHUNK, hipHostMallocDefault) != hipSuccess) return nullptr;
      chunks.push_back(c);
      for (int i = PER_CHUNK - 1; i >= 0; --i) free_.push_back((char*)c + (size_t)i * SLOT);
    }
    void* p = free_.back();
    free_.pop_back();
    return p;
  }
  void put(void* p) {
    if (p) free_.push_back(p);
  }
  void release_all() {
    for (void* c : chunks) hipHostFree(c);
    chunks.clear();
    free_.clear();
  }
};

struct fab_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  Arena arena;
  std::mutex mu;                 // arena + request table
  std::condition_variable cv;
  std::vector<hipStream_t> pool; // serving streams
  std::vector<int> pool_busy;
  int block_max = 32;            // largest block of merged single-rhs requests (1: no merging)
  bool hold = false;             // fab_hold: admit nothing while set
  // sampled SRHT rows per (padded length, s, seed), device arrays in the arena
  std::map<std::tuple<long long, int, uint64_t>, int*> srht_cache;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> reqs;
  uint64_t next_id = 1;
  std::thread sched;
  bool stop = false;
  std::set<fab_matrix> matrices;
  PinnedSlots pinned;            // requests' pinned info blocks and flags
  double* host_info = nullptr;   // pinned staging for blocking solves
  int* host_flag = nullptr;      // pinned: LSQR stop flag of blocking solves
  std::mutex solve_mu;
  Prof prof;
  // Replayable graphs of blocking solves, keyed by everything the launch
  // sequence depends on (plan, pointers, profiling mask); small LRU.
  struct GraphEntry {
    std::string key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<std::pair<int, size_t>> marks;   // profiling event pairs recorded in the graph
    size_t events_used = 0;
    unsigned long long last_use = 0;
  };
  std::vector<GraphEntry> graphs;
  unsigned long long graph_clock = 0;
  bool use_graphs = true;
};

namespace {

struct Request {
  uint64_t id = 0;
  Plan plan;
  char* ws = nullptr;
  int stream_idx = -1;
  hipEvent_t done_ev = nullptr;
  double* host_info = nullptr;   // pinned: [nrhs][NINFO] + status
  int state = 0;                 // 0 queued, 1 running, 2 done
  int status = FAB_OK;
  double t_submit = 0.0, t_done = 0.0;
  std::vector<fab_info> info;
  int fell_back = 0;             // recomputed with an FP64 basis (FAB_PREC_AUTO)
  int refined = 0;               // least-squares refinement enqueued
  // Blocked requests: single-rhs requests on the same resident matrix with
  // the same function and parameters run as the columns of one block solve
  // (nrhs = members.size()), a request of the library's own that gathers
  // their b into its workspace and scatters the columns of its result.
  std::vector<uint64_t> members;        // block: the user requests, column q = members[q]
  std::vector<const double*> mb;        // block: their b
  std::vector<double*> mout;            // block: their out
  uint64_t block = 0;                   // user request: the block that runs it (0: runs on its own)
  size_t oBlkB = 0, oBlkO = 0;          // block: interleaved b and result in the workspace
  // The launch sequence of each phase (the solve, then a refinement) is
  // issued by a worker thread of the request's own, so that the launches of
  // the requests on the pool streams are issued in parallel while the
  // scheduler keeps admitting and retiring; the whitened basis also reads
  // its trigger on the host every few steps in that thread.
  std::thread worker;
  std::atomic<bool> worker_done{false};
  int worker_rc = FAB_OK;
  int* flag_host = nullptr;             // pinned: flags the worker reads (whitening trigger, LSQR stop)
};

// Sampled SRHT rows for (npad, s, seed): computed once on `st` (which the
// caller then synchronises with) and cached in the arena.  Caller holds ctx->mu.
const int* srht_rows_cached(fab_ctx ctx, long long npad, int s, uint64_t seed, hipStream_t st, int* rc) {
  const auto key = std::make_tuple(npad, s, seed);
  auto it = ctx->srht_cache.find(key);
  if (it != ctx->srht_cache.end()) return it->second;
  int* rows = (int*)ctx->arena.alloc_high((size_t)s * 4);
  if (!rows) { *rc = FAB_ENOMEM; return nullptr; }
  if (srht_sample_rows(rows, npad, s, sm64_out(seed, 2), st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
    ctx->arena.release(rows);
    *rc = FAB_EDEVICE;
    return nullptr;
  }
  ctx->srht_cache[key] = rows;
  return rows;
}

constexpr size_t host_info_doubles(int nrhs) { return (size_t)nrhs * NINFO + 4 + 2 * nrhs + 8; }
static_assert(host_info_doubles(32) * 8 <= PinnedSlots::SLOT, "a pinned slot holds the info block of 32 rhs");

// Enqueue the whole solve on `st`.  Host-visible results land in `hinfo` (pinned).
// `side` runs the incremental sketched QR; `ev` orders it against `st`;
// `rows` holds the sampled SRHT rows (cached per context).
// Operator fields of a descriptor (the start vector of a sign-function solve).
SolveDev operator_desc(fab_matrix A, int nrhs) {
  SolveDev d{};
  d.n = A->n;
  d.nrhs = nrhs;
  d.lognrhs = ilog2(nrhs);
  d.op = A->op;
  d.prod = A->op == OP_CSR ? PROD_CSR : PROD_FUSED;
  d.nx = A->nx;
  d.ny = A->ny;
  d.nz = A->nz;
  for (int i = 0; i < 7; ++i) d.c[i] = A->c[i];
  d.rowptr = A->rowptr;
  d.col = A->col;
  d.val = A->val;
  return d;
}

// Kernel descriptors of a planned request in its workspace.
void build_descs(const Plan& P, char* ws, const int* rows, SolveDev& d, DenseDev& g) {
  const fab_params& p = P.p;
  fab_matrix A = P.A;
  const int m = p.m, s = p.s, nr = P.nrhs;
  d = SolveDev{};
  d.n = A->n;
  d.nrhs = nr;
  d.lognrhs = ilog2(nr);
  d.m = m;
  d.k = p.k;
  d.s = s;
  d.zeta = p.zeta;
  // a CSR matrix and the sign function's A^2 reach the streaming passes as
  // a product written to wbuf before them; a stencil alone is fused
  d.op = (A->op == OP_CSR || P.sign) ? OP_CSR : OP_STENCIL;
  d.prod = P.sign ? (A->op == OP_CSR ? PROD_SQ_CSR : PROD_SQ_STENCIL) : (A->op == OP_CSR ? PROD_CSR : PROD_FUSED);
  d.nx = A->nx;
  d.ny = A->ny;
  d.nz = A->nz;
  for (int i = 0; i < 7; ++i) d.c[i] = A->c[i];
  d.rowptr = A->rowptr;
  d.col = A->col;
  d.val = A->val;
  d.V = ws + P.oV;
  d.ldv = P.ldv;
  d.wbuf = d.op == OP_CSR ? (double*)(ws + P.oW) : nullptr;
  d.wtmp = P.sign ? (double*)(ws + P.oWtmp) : nullptr;
  d.b = P.sign ? (const double*)(ws + P.oSignB) : P.b;
  d.H = (double*)(ws + P.oH);
  d.eta = (double*)(ws + P.oEta);
  d.wnorm = (double*)(ws + P.oWn);
  d.coef = (double*)(ws + P.oCoef);
  d.S = (double*)(ws + P.oS);
  d.log_tile = P.LT;
  d.rows_per_tile = P.R;
  d.log_rows = P.logR;
  d.ntiles = P.ntiles;
  d.nblk = P.nblk;
  d.nred = P.nred;
  d.part = (double*)(ws + P.oPart);
  d.npart = (double*)(ws + P.oNpart);
  d.skpart = (double*)(ws + P.oSk);
  d.skstride = (((long long)p.s * nr + 7) & ~7LL) * P.nblk;
  d.counter = (unsigned*)(ws + P.oCnt);
  d.status = (int*)(ws + P.oStatus);
  d.sketch = p.sketch == FAB_SKETCH_SRHT ? SK_SRHT : SK_SPARSE;
  d.sk_slices = P.sk_slices;
  d.sk_reg = P.sk_reg;
  d.tgroups = P.tgroups;
  d.tchunk = ((long long)P.ntiles + P.tgroups - 1) / P.tgroups;
  d.wtp = P.wtp;
  d.wc = P.wc;
  d.wpen = P.wpen;
  d.wz = P.wz;
  d.srht_rows = rows;
  if (d.sketch == SK_SRHT) {
    d.key_a = sm64_out(p.seed, 1);
    d.key_b = 0;
    d.sk_scale = 1.0 / std::sqrt((double)s);
  } else {
    d.key_a = sm64_out(p.seed, 3);
    d.key_b = sm64_out(p.seed, 4);
    d.sk_scale = 1.0 / std::sqrt((double)p.zeta);
  }
  d.unit_round = P.esize == 4 ? std::ldexp(1.0, -24) : std::ldexp(1.0, -53);

  g = DenseDev{};
  g.m = m;
  g.s = s;
  g.nrhs = nr;
  g.stride = (long long)P.dense_stride;
  g.base = (double*)(ws + P.oDense);
  g.oW = (long long)P.oDW;
  g.oR = (long long)P.oDR;
  g.oH = (long long)P.oDH;
  g.oM = (long long)P.oDM;
  g.oVec = (long long)P.oDVec;
  g.oInfo = (long long)P.oDInfo;
  g.ls_mode = p.ls_mode == FAB_LS_NONE ? 2 : 1;
  g.nvar = P.nvar;
  g.unit_round = d.unit_round;
  g.fkind = P.f.kind;
  g.alpha = P.f.alpha;
  g.sigma = P.f.sigma;
  g.p = P.f.p;
  g.ncoef = (int)P.coef.size();
  for (size_t i = 0; i < P.coef.size(); ++i) g.coef[i] = P.coef[i];

}

int enqueue_solve(Plan& P, char* ws, hipStream_t st, const int* rows, double* hinfo, Prof* prof = nullptr,
                  int* host_flag = nullptr) {
  const int m = P.p.m, nr = P.nrhs;
  SolveDev d;
  DenseDev g;
  build_descs(P, ws, rows, d, g);
  hipError_t e;
  // zero the small state: H, eta, wnorm, coef, S, counter, status (contiguous from oH .. oRows)
  if ((e = zero_fill(ws + P.oH, P.oPart - P.oH, st)) != hipSuccess) return FAB_EDEVICE;
  if ((e = zero_fill(ws + P.oCnt, P.oRows - P.oCnt, st)) != hipSuccess) return FAB_EDEVICE;
  int open_cls = -1;
  auto B = [&](int cls) {
    if (prof && (prof->mask >> cls) & 1) { prof->begin(cls, st); open_cls = cls; }
  };
  auto E = [&]() {
    if (open_cls >= 0) { prof->end(st); open_cls = -1; }
  };
  if (P.sign) {
    // start vector A b of the solve on A^2
    SolveDev da = operator_desc(P.A, P.nrhs);
    B(FAB_K_OTHER);
    e = apply_operator(da, P.b, (double*)(ws + P.oSignB), st);
    E();
    if (e != hipSuccess) return FAB_EDEVICE;
  }
  B(FAB_K_OTHER);
  e = basis_start(d, P.esize, st, P.lds_kupdate);
  E();
  if (e != hipSuccess) return FAB_EDEVICE;
  if (P.bg) {
    double* bcf = (double*)(ws + P.oBgCf);
    for (int i = 0; i <= m && e == hipSuccess; ++i) {
      if (i > 0) {
        B(FAB_K_DOTS);
        e = bg_apply(d, P.esize, i, st, P.lds_update);
        E();
        if (e != hipSuccess) break;
      }
      B(FAB_K_OTHER);
      e = bg_reduce(d, i, st);
      if (e == hipSuccess) e = bg_gs(d, bcf, i, P.p.basis == FAB_BASIS_SKETCHED_GS2 ? 2 : 1, st);
      E();
      if (e != hipSuccess || i == 0) continue;
      B(FAB_K_UPDATE);
      e = bg_update(d, P.esize, bcf, i, st);
      E();
    }
    if (e != hipSuccess) return FAB_EDEVICE;
  }
  // Truncated basis.  With whitening, after the update pass of step i the
  // newest sketch column joins the condition monitor; every WH_EVERY steps
  // the host reads the trigger, and on a trigger step i is discarded, the
  // basis V_i is whitened and steps i..m follow Algorithm 1.
  P.whitened_at = 0;
  int* wflag = P.whiten ? (int*)(ws + P.oWflag) : nullptr;
  if (P.whiten && (!host_flag || zero_fill(wflag, 256, st) != hipSuccess)) return FAB_EDEVICE;
  for (int i = 1; i <= m && !P.bg && !P.whitened_at; ++i) {
    B(FAB_K_DOTS);
    e = basis_dots(d, P.esize, i, st);
    E();
    if (e != hipSuccess) return FAB_EDEVICE;
    B(FAB_K_UPDATE);
    e = basis_update(d, P.esize, i, st, P.lds_kupdate);
    E();
    if (e != hipSuccess) return FAB_EDEVICE;
    if (!P.whiten) continue;
    const int check = (i % WH_EVERY == 0 && i >= 2) ? 1 : 0;
    B(FAB_K_OTHER);
    e = wh_col(d, g, i - 1, check, WH_THRESH, wflag, st);
    E();
    if (e != hipSuccess) return FAB_EDEVICE;
    if (!check) continue;
    *host_flag = 0;
    if (hipMemcpyAsync(host_flag, wflag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return FAB_EDEVICE;
    if (!*host_flag) continue;
    P.whitened_at = i;
    // an FP32 basis whitened here carries up to 2^-24 kappa(R) > 2^-24
    // WH_THRESH of rounding (the bound collect_info reports): when that
    // alone fails the FP64 rerun test, the rest of this attempt is wasted
    if (P.p.prec == FAB_PREC_AUTO && P.esize == 4 && !(std::ldexp(1.0, -24) * WH_THRESH <= P.p.tol / 2))
      return RC_RERUN_FP64;
    B(FAB_K_OTHER);
    e = wh_whiten(d, g, P.esize, i, st);
    E();
    if (e != hipSuccess) return FAB_EDEVICE;
    double* bcf = (double*)(ws + P.oBgCf);
    for (int j = i; j <= m && e == hipSuccess; ++j) {
      B(FAB_K_DOTS);
      e = bg_apply(d, P.esize, j, st, P.lds_update);
      E();
      if (e != hipSuccess) break;
      B(FAB_K_OTHER);
      e = bg_reduce(d, j, st);
      if (e == hipSuccess) e = bg_gs(d, bcf, j, 1, st);
      E();
      if (e != hipSuccess) break;
      B(FAB_K_UPDATE);
      e = bg_update(d, P.esize, bcf, j, st);
      E();
    }
    if (e != hipSuccess) return FAB_EDEVICE;
  }
  if (!P.bg && !P.whitened_at) {
    B(FAB_K_OTHER);
    e = basis_finish(d, P.esize, st);
    E();
    if (e != hipSuccess) return FAB_EDEVICE;
  }
  double* cf = (double*)(ws + P.oCf);
  B(FAB_K_DENSE);
  e = dense_tail(d, g, cf, (double*)(ws + P.oFq), st);
  E();
  if (e != hipSuccess) return FAB_EDEVICE;
  B(FAB_K_COMBINE);
  e = basis_combine(d, P.esize, cf, m, P.out, st);
  E();
  if (e != hipSuccess) return FAB_EDEVICE;
  // results to pinned host memory: per-rhs dense info, then status ints
  for (int q = 0; q < nr; ++q) {
    e = hipMemcpyAsync(hinfo + (size_t)q * NINFO, g.base + (size_t)q * P.dense_stride + P.oDInfo, NINFO * 8,
                       hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return FAB_EDEVICE;
  }
  e = hipMemcpyAsync(hinfo + (size_t)nr * NINFO, d.status, (size_t)(4 + 2 * nr) * 4, hipMemcpyDeviceToHost, st);
  if (e != hipSuccess) return FAB_EDEVICE;
  return FAB_OK;
}

int collect_info(const Plan& P, const double* hinfo, std::vector<fab_info>& out) {
  const int nr = P.nrhs;
  const int* status = (const int*)(hinfo + (size_t)nr * NINFO);
  out.assign(nr, fab_info{});
  int rc = FAB_OK;
  if (status[1]) rc = FAB_ENUMERIC;
  for (int q = 0; q < nr; ++q) {
    const double* in = hinfo + (size_t)q * NINFO;
    fab_info& fi = out[q];
    fi.m_used = status[4 + 2 * q];
    fi.breakdown = status[5 + 2 * q] ? 1 : 0;
    fi.kappa_R = in[0];
    fi.h_last = in[1];
    fi.beta = in[2];
    fi.prec_used = P.esize == 4 ? FAB_PREC_FP32 : FAB_PREC_FP64;
    if (P.nvar == 3) {
      fi.ls_gate = in[INFO_GATE];
      fi.round_est = in[INFO_ROUND];
      fi.conv_est = in[INFO_CONV];
      fi.err_est = std::max(fi.ls_gate, fi.round_est);
    } else {
      fi.err_est = fi.ls_gate = fi.round_est = fi.conv_est = 0.0;
    }
    fi.ls_iters = (int)in[INFO_LSQR_IT];
    fi.ls_limit = in[INFO_LSQR_LIMIT] != 0.0 ? 1 : 0;
    // refined: the least-squares part of the error is the Paige-Saunders
    // measure of the last LSQR iteration (a backward error of the least
    // squares; zero after the exact solve through the Gram matrix, which is
    // only accepted when kappa(R)^2 u <= tol / 10)
    if (fi.ls_iters > 0) fi.err_est = std::max(in[INFO_LSQR_RATIO], fi.round_est);
    if (P.gram_used) fi.err_est = fi.round_est;
    // a whitened FP32 basis: the transform V R^{-1} multiplies the storage
    // rounding of the vectors it whitens by up to kappa(R), which exceeded
    // WH_THRESH when it triggered (Section 2.1.2); the rounding estimate,
    // first order in the final basis, does not see that, so the bound is
    // added (with or without the automatic policies)
    if (P.whitened_at && P.esize == 4) {
      fi.round_est = std::max(fi.round_est, std::ldexp(1.0, -24) * WH_THRESH);
      fi.err_est = std::max(fi.err_est, fi.round_est);
    }
    fi.fell_back = 0;
    fi.whitened_at = P.whitened_at;
    fi.block_rhs = 1;
    if (in[3] != 0.0) rc = FAB_ENUMERIC;
    if (!std::isfinite(fi.beta)) rc = FAB_ENUMERIC;
  }
  return rc;
}

int esize_for(int prec) { return prec == FAB_PREC_FP64 ? 8 : 4; }

// LSQR refinement of the least squares (FAB_LS_LSQR always; FAB_LS_AUTO when
// the gate ||R (c_y - c_0)|| / ||R c_y|| exceeds tol/10, or always with a
// sketched Gram-Schmidt basis), then f, the estimates, the weights and the
// combination again, and the info copy.  With `host_flag` (pinned; blocking
// solves) the iterations are issued in chunks and the stream is synchronised
// after each to stop issuing once every right-hand side has stopped; without
// it (served requests) the whole fixed-length sequence is enqueued.  Both
// stop at the same iteration: the device flag decides.
int enqueue_refine(Plan& P, char* ws, hipStream_t st, const int* rows, double* hinfo, int* host_flag = nullptr) {
  SolveDev d;
  DenseDev g;
  build_descs(P, ws, rows, d, g);
  LsqrDev L{};
  L.u = (double*)(ws + P.oLu);
  L.part = (double*)(ws + P.oLpart);
  L.st = (double*)(ws + P.oLst);
  L.stride = (long long)lsqr_state_stride(P.p.m);
  L.alldone = (int*)(ws + P.oLflag);
  L.rinv = (double*)(ws + P.oLri);
  L.nblk = P.lnblk;
  L.maxit = P.p.ls_maxit > 0 ? P.p.ls_maxit : ((P.bg || P.whitened_at) ? 128 : 32);
  L.tol = P.p.tol / 10;
  if (zero_fill(ws + P.oLflag, 256, st) != hipSuccess) return FAB_EDEVICE;
  // FAB_LS_GRAM (blocking calls): the exact solve through the Gram matrix;
  // LSQR below when its factorisation is not usable
  P.gram_used = false;
  if (P.gram && host_flag) {
    int* gflag = (int*)(ws + P.oGflag);
    if (gram_ls_launch(d, g, (double*)(ws + P.oGpart), gflag, P.esize, P.p.tol, st) != hipSuccess)
      return FAB_EDEVICE;
    *host_flag = 1;
    if (hipMemcpyAsync(host_flag, gflag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return FAB_EDEVICE;
    P.gram_used = *host_flag == 0;
  }
  if (P.gram_used) {
    // y and H_hat are in place; nothing to iterate
  } else if (!host_flag) {
    if (lsqr_launch(d, g, L, P.esize, st) != hipSuccess) return FAB_EDEVICE;
  } else {
    // chunks of 2, 4, 8, then 16 iterations: a refinement that stops after
    // an iteration or two issues few launches past its end
    if (lsqr_begin(d, g, L, P.esize, st) != hipSuccess) return FAB_EDEVICE;
    for (int it = 0, chunk = 2; it < L.maxit; it += chunk, chunk = std::min(2 * chunk, 16)) {
      if (lsqr_iterate(d, g, L, P.esize, st, std::min(chunk, L.maxit - it)) != hipSuccess) return FAB_EDEVICE;
      *host_flag = 0;
      if (hipMemcpyAsync(host_flag, L.alldone, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return FAB_EDEVICE;
      if (*host_flag) break;
    }
    if (lsqr_end(d, g, L, st) != hipSuccess) return FAB_EDEVICE;
  }
  double* cf = (double*)(ws + P.oCf);
  if (dense_after_refine(d, g, cf, (double*)(ws + P.oFq), st) != hipSuccess) return FAB_EDEVICE;
  if (basis_combine(d, P.esize, cf, P.p.m, P.out, st) != hipSuccess) return FAB_EDEVICE;
  const int nr = P.nrhs;
  for (int q = 0; q < nr; ++q)
    if (hipMemcpyAsync(hinfo + (size_t)q * NINFO, g.base + (size_t)q * P.dense_stride + P.oDInfo, NINFO * 8,
                       hipMemcpyDeviceToHost, st) != hipSuccess)
      return FAB_EDEVICE;
  if (hipMemcpyAsync(hinfo + (size_t)nr * NINFO, d.status, (size_t)(4 + 2 * nr) * 4, hipMemcpyDeviceToHost, st) !=
      hipSuccess)
    return FAB_EDEVICE;
  return FAB_OK;
}

bool needs_refine(const Plan& P, int rc, const std::vector<fab_info>& fi) {
  if (rc != FAB_OK || !P.lsqr) return false;
  if (P.p.ls_mode == FAB_LS_LSQR || P.p.ls_mode == FAB_LS_GRAM || P.bg || P.whitened_at) return true;
  for (const auto& x : fi)
    if (!x.breakdown && !(x.ls_gate <= P.p.tol / 10)) return true;
  return false;
}

// FAB_PREC_AUTO: an FP32-basis result is recomputed with an FP64 basis when
// the basis-rounding estimate exceeds tol/2 or the FP32 run produced
// non-finite values.  Decided once, on the solve's own result (before any
// least-squares refinement), in blocking and served calls alike.  The
// estimate overestimates the rounding error (first-order bound), and a
// refinement stops at a least-squares measure of tol/10, so an accepted
// result stays below tol.
bool needs_fp64_rerun(const Plan& P, int rc, const std::vector<fab_info>& fi) {
  if (P.p.prec != FAB_PREC_AUTO || P.esize != 4) return false;
  if (rc == FAB_ENUMERIC) return true;
  if (rc != FAB_OK) return false;
  for (const auto& x : fi)
    if (!(x.round_est <= P.p.tol / 2)) return true;
  return false;
}

// ---------------------------------------------------------------- scheduler
// The caller's function of a plan (the sign function plans the inverse
// square root; a polynomial's coefficients are the plan's own copy).
fab_func plan_func(const Plan& P) {
  fab_func f = P.sign ? P.forig : P.f;
  if (f.kind == FAB_F_POLY) f.coef = P.coef.data();
  return f;
}

// Workspace of a block: the plan's, then the interleaved b and result.
void add_block_buffers(Request& r) {
  const size_t nb = align256((size_t)r.plan.A->n * r.plan.nrhs * 8);
  r.oBlkB = align256(r.plan.bytes);
  r.oBlkO = r.oBlkB + nb;
  r.plan.bytes = r.oBlkO + nb;
}

// Copy the block's result columns to the member requests' out.
hipError_t scatter_block(const Request& r, hipStream_t st) {
  OutPtrs o{};
  for (size_t q = 0; q < r.mout.size(); ++q) o.p[q] = r.mout[q];
  return scatter_cols((const double*)(r.ws + r.oBlkO), ilog2(r.plan.nrhs), r.plan.A->n, o, st);
}

void retire_locked(fab_ctx ctx, Request& r) {
  if (r.worker.joinable()) r.worker.join();
  const bool blk = !r.members.empty();
  const bool stopped = r.worker_rc == RC_RERUN_FP64;   // FP32 attempt stopped at its whitening
  if (r.worker_rc != FAB_OK && !stopped) {
    // the worker could not issue the phase: wait for what it did issue, then
    // complete the request (or the block's members) with its error
    hipStreamSynchronize(ctx->pool[r.stream_idx]);
    r.status = r.worker_rc;
  } else if (stopped) {
    r.status = FAB_ENOMEM;   // unless the FP64 rerun below is queued
    r.info.assign(r.plan.nrhs, fab_info{});
  } else {
    r.status = collect_info(r.plan, r.host_info, r.info);
  }
  // the precision decision is taken on the solve's result, as in blocking
  // calls (a refinement's result is not judged again)
  if ((stopped || (r.worker_rc == FAB_OK && needs_fp64_rerun(r.plan, r.status, r.info))) && !r.fell_back &&
      !r.refined) {
    // FAB_PREC_AUTO: queue the request again, first in line, with an FP64 basis
    Plan P2;
    const fab_func f2 = plan_func(r.plan);
    if (make_plan(r.plan.A, r.plan.nrhs, f2, &r.plan.p, 8, P2) == FAB_OK &&
        ctx->arena.could_ever_fit(P2.bytes + (blk ? 2 * align256((size_t)r.plan.A->n * r.plan.nrhs * 8) + 256 : 0))) {
      P2.b = r.plan.b;
      P2.out = r.plan.out;
      ctx->arena.release(r.ws);
      r.ws = nullptr;
      ctx->pool_busy[r.stream_idx] = 0;
      r.plan = P2;
      if (blk) add_block_buffers(r);
      r.fell_back = 1;
      r.state = 0;
      ctx->queue.push_front(r.id);
      return;
    }
  }
  if (r.worker_rc == FAB_OK && !r.refined && needs_refine(r.plan, r.status, r.info)) {
    // least-squares refinement on the request's stream, issued by a worker
    // as the solve was; retired when it ends
    r.refined = 1;
    Request* rp = &r;
    const int dev = ctx->device;
    const hipStream_t st = ctx->pool[r.stream_idx];
    r.worker_done.store(false);
    r.worker_rc = FAB_OK;
    r.worker = std::thread([rp, dev, st, blk]() {
      hipSetDevice(dev);
      // the worker may wait: it issues the iterations in chunks and stops
      // once the device flag says every rhs stopped, as blocking calls do
      int wrc = enqueue_refine(rp->plan, rp->ws, st, nullptr, rp->host_info, rp->flag_host);
      if (wrc == FAB_OK && blk && scatter_block(*rp, st) != hipSuccess) wrc = FAB_EDEVICE;
      if (wrc == FAB_OK && hipEventRecord(rp->done_ev, st) != hipSuccess) wrc = FAB_EDEVICE;
      rp->worker_rc = wrc;
      rp->worker_done.store(true);
    });
    return;
  }
  if (r.fell_back)
    for (auto& fi : r.info) fi.fell_back = 1;
  r.t_done = now_us();
  ctx->arena.release(r.ws);
  r.ws = nullptr;
  ctx->pool_busy[r.stream_idx] = 0;
  if (!blk) {
    for (auto& fi : r.info) fi.latency_us = r.t_done - r.t_submit;
    r.plan.A->refs.fetch_sub(1);
    r.state = 2;
    return;
  }
  // a block: each member request gets its column's record and completes
  for (size_t q = 0; q < r.members.size(); ++q) {
    auto it = ctx->reqs.find(r.members[q]);
    if (it == ctx->reqs.end()) continue;
    Request& u = *it->second;
    u.info.assign(1, q < r.info.size() ? r.info[q] : fab_info{});
    u.info[0].block_rhs = (int)r.members.size();
    u.status = r.status;
    u.t_done = r.t_done;
    u.info[0].latency_us = u.t_done - u.t_submit;
    u.fell_back = r.fell_back;
    u.block = 0;
    u.plan.A->refs.fetch_sub(1);
    u.state = 2;
  }
  r.state = 3;   // the block itself is dropped by the scheduler
}

// Single-rhs requests that can run as columns of one block solve: the same
// resident matrix, function and parameters, the sketch seed included, so that
// every column uses the sketch it would use alone.
bool blockable(const Request& r) {
  return r.members.empty() && r.block == 0 && r.plan.nrhs == 1 && !r.fell_back && !r.plan.whiten;
}
bool same_solve(const Plan& a, const Plan& b) {
  const fab_func fa = plan_func(a), fb = plan_func(b);
  if (a.A != b.A || a.esize != b.esize || a.sign != b.sign) return false;
  if (fa.kind != fb.kind || fa.alpha != fb.alpha || fa.sigma != fb.sigma || fa.p != fb.p || a.coef != b.coef)
    return false;
  const fab_params &p = a.p, &q = b.p;
  return p.m == q.m && p.k == q.k && p.s == q.s && p.sketch == q.sketch && p.zeta == q.zeta && p.seed == q.seed &&
         p.prec == q.prec && p.ls_mode == q.ls_mode && p.tol == q.tol && p.basis == q.basis &&
         p.ls_maxit == q.ls_maxit;
}

// Merge the queued single-rhs requests compatible with `head` (in queue
// order, at most block_max, a power of two >= 2 of them) into a block placed
// at the front of the queue.  Returns false when there is nothing to merge.
bool form_block_locked(fab_ctx ctx, const Request& head) {
  std::vector<uint64_t> ids;
  for (uint64_t id : ctx->queue) {
    auto jt = ctx->reqs.find(id);
    if (jt == ctx->reqs.end()) continue;
    if (blockable(*jt->second) && same_solve(jt->second->plan, head.plan)) {
      ids.push_back(id);
      if ((int)ids.size() >= ctx->block_max) break;
    }
  }
  int g = 1;
  while (2 * g <= (int)ids.size() && 2 * g <= 32) g *= 2;
  // the largest such block that can fit the arena at all
  auto b = std::make_shared<Request>();
  for (; g >= 2; g /= 2) {
    if (make_plan(head.plan.A, g, plan_func(head.plan), &head.plan.p, head.plan.esize, b->plan) != FAB_OK) return false;
    add_block_buffers(*b);
    if (ctx->arena.could_ever_fit(b->plan.bytes)) break;
  }
  if (g < 2) return false;
  ids.resize(g);
  if (hipEventCreateWithFlags(&b->done_ev, hipEventDisableTiming) != hipSuccess) return false;
  if (!(b->host_info = (double*)ctx->pinned.get())) {
    hipEventDestroy(b->done_ev);
    b->done_ev = nullptr;
    return false;
  }
  b->id = ctx->next_id++;
  b->t_submit = now_us();
  for (uint64_t id : ids) {
    Request& u = *ctx->reqs[id];
    b->members.push_back(id);
    b->mb.push_back(u.plan.b);
    b->mout.push_back(u.plan.out);
    u.block = b->id;
    u.state = 1;
    b->t_submit = std::min(b->t_submit, u.t_submit);
  }
  std::deque<uint64_t> rest;
  for (uint64_t id : ctx->queue)
    if (std::find(ids.begin(), ids.end(), id) == ids.end()) rest.push_back(id);
  rest.push_front(b->id);
  ctx->queue.swap(rest);
  ctx->reqs[b->id] = b;
  return true;
}

void admit_locked(fab_ctx ctx) {
  while (!ctx->hold && !ctx->queue.empty()) {
    auto it = ctx->reqs.find(ctx->queue.front());
    if (it == ctx->reqs.end()) { ctx->queue.pop_front(); continue; }
    int si = -1;
    for (size_t i = 0; i < ctx->pool.size(); ++i)
      if (!ctx->pool_busy[i]) { si = (int)i; break; }
    if (si < 0) return;
    // continuous batching: queued single-rhs requests on the same matrix
    // with the same function and parameters become one block solve
    if (ctx->block_max >= 2 && blockable(*it->second) && form_block_locked(ctx, *it->second)) continue;
    Request& r = *it->second;
    const bool blk = !r.members.empty();
    char* ws = (char*)ctx->arena.alloc(r.plan.bytes);
    if (!ws) return;   // FIFO: wait until running requests free memory
    ctx->queue.pop_front();
    r.ws = ws;
    r.stream_idx = si;
    ctx->pool_busy[si] = 1;
    hipSetDevice(ctx->device);
    const hipStream_t st = ctx->pool[si];
    int rc = FAB_OK;
    if (blk) {
      r.plan.b = (const double*)(ws + r.oBlkB);
      r.plan.out = (double*)(ws + r.oBlkO);
      ColPtrs c{};
      for (size_t q = 0; q < r.mb.size(); ++q) c.p[q] = r.mb[q];
      if (gather_cols(c, ilog2(r.plan.nrhs), r.plan.A->n, (double*)(ws + r.oBlkB), st) != hipSuccess) rc = FAB_EDEVICE;
    }
    const int* rows = nullptr;
    if (rc == FAB_OK && r.plan.p.sketch == FAB_SKETCH_SRHT)
      rows = srht_rows_cached(ctx, 1LL << ilog2(r.plan.A->n), r.plan.p.s, r.plan.p.seed, st, &rc);
    if (rc == FAB_OK) {
      // the worker issues the sequence (a whitened basis reads its trigger on
      // the host meanwhile) and records done_ev; the scheduler retires the
      // request after both.  Only the worker touches r.plan until then.
      Request* rp = &r;
      const int dev = ctx->device;
      r.worker_done.store(false);
      r.worker_rc = FAB_OK;
      r.worker = std::thread([rp, dev, st, rows, ws, blk]() {
        hipSetDevice(dev);
        int wrc = enqueue_solve(rp->plan, ws, st, rows, rp->host_info, nullptr,
                                rp->plan.whiten ? rp->flag_host : nullptr);
        if (wrc == FAB_OK && blk && scatter_block(*rp, st) != hipSuccess) wrc = FAB_EDEVICE;
        if ((wrc == FAB_OK || wrc == RC_RERUN_FP64) && hipEventRecord(rp->done_ev, st) != hipSuccess)
          wrc = FAB_EDEVICE;
        rp->worker_rc = wrc;
        rp->worker_done.store(true);
      });
      r.state = 1;
      continue;
    }
    {
      hipStreamSynchronize(st);
      ctx->arena.release(ws);
      r.ws = nullptr;
      ctx->pool_busy[si] = 0;
      r.status = rc;
      r.t_done = now_us();
      if (!blk) {
        r.plan.A->refs.fetch_sub(1);
        r.state = 2;
        continue;
      }
      for (uint64_t id : r.members) {
        auto jt = ctx->reqs.find(id);
        if (jt == ctx->reqs.end()) continue;
        Request& u = *jt->second;
        u.status = rc;
        u.t_done = r.t_done;
        u.block = 0;
        u.plan.A->refs.fetch_sub(1);
        u.state = 2;
      }
      r.state = 3;
    }
  }
}

// Drop finished blocks (their members carry the results).
void drop_blocks_locked(fab_ctx ctx) {
  for (auto it = ctx->reqs.begin(); it != ctx->reqs.end();) {
    if (it->second->state == 3) {
      if (it->second->done_ev) hipEventDestroy(it->second->done_ev);
      ctx->pinned.put(it->second->host_info);
      it = ctx->reqs.erase(it);
    } else {
      ++it;
    }
  }
}

void scheduler_main(fab_ctx ctx) {
  hipSetDevice(ctx->device);
  std::unique_lock<std::mutex> lk(ctx->mu);
  while (true) {
    bool progressed = false;
    for (auto& kv : ctx->reqs) {
      Request& r = *kv.second;
      // members of a block complete with their block
      if (r.state == 1 && r.block == 0 && (!r.worker.joinable() || r.worker_done.load()) &&
          hipEventQuery(r.done_ev) == hipSuccess) {
        retire_locked(ctx, r);
        progressed = true;
      }
    }
    admit_locked(ctx);
    drop_blocks_locked(ctx);
    if (progressed) ctx->cv.notify_all();
    bool running = false;
    for (auto& kv : ctx->reqs)
      if (kv.second->state == 1) running = true;
    if (ctx->stop && !running && ctx->queue.empty()) break;
    if (running) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else {
      ctx->cv.wait_for(lk, std::chrono::milliseconds(5));
    }
  }
}

}  // namespace

// ============================================================== C ABI
extern "C" {

const char* fab_version(void) { return "libfab 0.1 (gfx950)"; }

const char* fab_strerror(int code) {
  switch (code) {
    case FAB_OK: return "ok";
    case FAB_EINVAL: return "invalid argument";
    case FAB_ENOMEM: return "request can never fit the arena";
    case FAB_EDEVICE: return "HIP runtime error";
    case FAB_ENUMERIC: return "non-finite input or result";
    case FAB_EBUSY: return "matrix in use by in-flight requests";
    case FAB_ENOTFOUND: return "unknown request";
    case FAB_ESCRATCH: return "request exceeds the static scratch of fab_solve_noalloc";
    default: return "unknown status";
  }
}

int fab_init(fab_ctx* out, int device, void* arena_dev_ptr, size_t arena_bytes, void* hip_stream) {
  if (!out || arena_bytes < (1u << 20)) return FAB_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FAB_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return FAB_EDEVICE;
  // Raising the dynamic-LDS limit is best effort: a launch that needs more than
  // the device grants fails with a HIP error, reported as FAB_EDEVICE.
  (void)basis_set_attributes();
  (void)hipGetLastError();
  auto* ctx = new fab_ctx_s();
  ctx->device = device;
  char* base = (char*)arena_dev_ptr;
  if (!base) {
    if (hipMalloc((void**)&base, arena_bytes) != hipSuccess) { delete ctx; return FAB_EDEVICE; }
    ctx->arena.owned = true;
  }
  ctx->arena.init(base, arena_bytes);
  if (hip_stream) {
    ctx->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) { delete ctx; return FAB_EDEVICE; }
    ctx->own_stream = true;
  }
  (void)dense_set_attributes();
  (void)lsqr_set_attributes();
  (void)bg_set_attributes();
  (void)wh_set_attributes();
  (void)fsqrt_set_attributes();
  (void)hipGetLastError();
  if (noalloc_setup(device) != FAB_OK) {
    delete ctx;
    return FAB_EDEVICE;
  }
  // serving streams: FAB_SERVING_STREAMS (1..16), default 12; each runs one
  // admitted request at a time and should have a hardware queue of its own
  int npool = 12;
  if (const char* ev = std::getenv("FAB_SERVING_STREAMS")) {
    const int v = std::atoi(ev);
    if (v >= 1 && v <= 16) npool = v;
  }
  for (int i = 0; i < npool; ++i) {
    hipStream_t s;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      delete ctx;
      return FAB_EDEVICE;
    }
    ctx->pool.push_back(s);
    ctx->pool_busy.push_back(0);
  }
  if (hipHostMalloc((void**)&ctx->host_info, host_info_doubles(32) * 8, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&ctx->host_flag, 256, hipHostMallocDefault) != hipSuccess) {
    delete ctx;
    return FAB_EDEVICE;
  }
  if (const char* ev = std::getenv("FAB_NO_GRAPH")) ctx->use_graphs = ev[0] == '0';
  ctx->sched = std::thread(scheduler_main, ctx);
  *out = ctx;
  return FAB_OK;
}

int fab_create_matrix_stencil(fab_ctx ctx, int dim, int nx, int ny, int nz, const double coeff[7], fab_matrix* A) {
  if (!ctx || !A || !coeff) return FAB_EINVAL;
  if (dim != 2 && dim != 3) return FAB_EINVAL;
  if (nx < 1 || ny < 1 || nz < 1 || (dim == 2 && nz != 1)) return FAB_EINVAL;
  const long long n = (long long)nx * ny * nz;
  if (n >= (1LL << 31) || n < 2) return FAB_EINVAL;
  auto* M = new fab_matrix_s();
  M->ctx = ctx;
  M->op = OP_STENCIL;
  M->dim = dim;
  M->nx = nx;
  M->ny = ny;
  M->nz = nz;
  for (int i = 0; i < 7; ++i) M->c[i] = coeff[i];
  if (dim == 2) M->c[5] = M->c[6] = 0.0;
  M->n = (int)n;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->matrices.insert(M);
  }
  *A = M;
  return FAB_OK;
}

int fab_create_matrix_csr(fab_ctx ctx, int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* col,
                          const float* val, int ptr_is_device, fab_matrix* A) {
  if (!ctx || !A || !rowptr || n < 2 || n >= (1LL << 31) || nnz < 0 || nnz >= (1LL << 31)) return FAB_EINVAL;
  if (nnz > 0 && (!col || !val)) return FAB_EINVAL;
  hipSetDevice(ctx->device);
  std::vector<int32_t> hrp;
  if (!ptr_is_device) {
    if (rowptr[0] != 0 || rowptr[n] != nnz) return FAB_EINVAL;
    for (int64_t i = 0; i < n; ++i)
      if (rowptr[i + 1] < rowptr[i]) return FAB_EINVAL;
    for (int64_t i = 0; i < nnz; ++i)
      if (col[i] < 0 || col[i] >= n) return FAB_EINVAL;
  } else {
    // device input: bring the index arrays to the host once and validate them
    // the same way, so that no kernel ever gathers through a bad index
    hrp.resize(n + 1);
    std::vector<int32_t> hcol((size_t)nnz);
    if (hipMemcpy(hrp.data(), rowptr, (n + 1) * 4, hipMemcpyDeviceToHost) != hipSuccess) return FAB_EDEVICE;
    if (nnz > 0 && hipMemcpy(hcol.data(), col, nnz * 4, hipMemcpyDeviceToHost) != hipSuccess) return FAB_EDEVICE;
    if (hrp[0] != 0 || hrp[n] != nnz) return FAB_EINVAL;
    for (int64_t i = 0; i < n; ++i)
      if (hrp[i + 1] < hrp[i]) return FAB_EINVAL;
    for (int64_t i = 0; i < nnz; ++i)
      if (hcol[i] < 0 || hcol[i] >= n) return FAB_EINVAL;
  }
  const size_t brp = align256((size_t)(n + 1) * 4), bcol = align256((size_t)nnz * 4), bval = align256((size_t)nnz * 4);
  char* mem;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    mem = (char*)ctx->arena.alloc_high(brp + bcol + bval);
  }
  if (!mem) return FAB_ENOMEM;
  const hipMemcpyKind kind = ptr_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (hipMemcpy(mem, rowptr, (n + 1) * 4, kind) != hipSuccess ||
      (nnz > 0 && hipMemcpy(mem + brp, col, nnz * 4, kind) != hipSuccess) ||
      (nnz > 0 && hipMemcpy(mem + brp + bcol, val, nnz * 4, kind) != hipSuccess)) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->arena.release(mem);
    return FAB_EDEVICE;
  }
  auto* M = new fab_matrix_s();
  M->ctx = ctx;
  M->op = OP_CSR;
  M->n = (int)n;
  M->nnz = nnz;
  M->rowptr = (int*)mem;
  M->col = (int*)(mem + brp);
  M->val = (float*)(mem + brp + bcol);
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->matrices.insert(M);
  }
  *A = M;
  return FAB_OK;
}

namespace {

// Release a matrix's graphs, memory and registration (callers hold solve_mu and mu).
void release_matrix_locked(fab_ctx ctx, fab_matrix A) {
  for (auto it = ctx->graphs.begin(); it != ctx->graphs.end();) {
    fab_matrix gA;
    std::memcpy(&gA, it->key.data(), sizeof(gA));
    if (gA == A) {
      hipGraphExecDestroy(it->exec);
      hipGraphDestroy(it->graph);
      it = ctx->graphs.erase(it);
    } else {
      ++it;
    }
  }
  if (A->op == OP_CSR) ctx->arena.release(A->rowptr);
  ctx->matrices.erase(A);
  delete A;
}

}  // namespace

int fab_destroy_matrix(fab_matrix A) {
  if (!A) return FAB_EINVAL;
  fab_ctx ctx = A->ctx;
  // lock order everywhere: solve_mu, then mu
  std::lock_guard<std::mutex> slk(ctx->solve_mu);
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (A->refs.load() > 0) return FAB_EBUSY;
  release_matrix_locked(ctx, A);
  return FAB_OK;
}

static std::string graph_key(const Plan& P, const char* ws, const int* rows, const double* hinfo, int prof_mask,
                             const fab_func& f) {
  std::string k;
  auto put = [&](const void* x, size_t n) { k.append((const char*)x, n); };
  const void* ptrs[6] = {P.A, ws, P.b, P.out, rows, hinfo};
  put(ptrs, sizeof(ptrs));
  put(&P.nrhs, sizeof(int));
  put(&P.esize, sizeof(int));
  put(&P.p, sizeof(fab_params));
  put(&prof_mask, sizeof(int));
  put(&f.kind, sizeof(int));
  put(&f.alpha, sizeof(double));
  put(&f.sigma, sizeof(double));
  put(&f.p, sizeof(double));
  if (!P.coef.empty()) put(P.coef.data(), P.coef.size() * sizeof(double));
  return k;
}

// Enqueue one blocking solve on ctx->stream: replay a cached graph of the
// identical launch sequence when there is one, else capture (fork/join with
// the side stream included) and instantiate it, falling back to direct
// launches if capture is unavailable.
static int launch_solve(fab_ctx ctx, Plan& P, char* ws, const int* rows, const fab_func& f) {
  Prof* prof = ctx->prof.mask ? &ctx->prof : nullptr;
  // event pairs recorded inside a replayed graph do not time the kernels, so
  // timed (profiled) solves use direct launches of the same kernels
  // whitening reads its trigger on the host during the solve: direct launches
  if (!ctx->use_graphs || prof || P.whiten)
    return enqueue_solve(P, ws, ctx->stream, rows, ctx->host_info, prof, ctx->host_flag);
  const std::string key = graph_key(P, ws, rows, ctx->host_info, ctx->prof.mask, f);
  for (auto& g : ctx->graphs) {
    if (g.key == key) {
      g.last_use = ++ctx->graph_clock;
      if (prof) {
        prof->marks = g.marks;
        prof->used = g.events_used;
      }
      return hipGraphLaunch(g.exec, ctx->stream) == hipSuccess ? FAB_OK : FAB_EDEVICE;
    }
  }
  if (prof) {
    // make sure every event the capture will use already exists
    while (prof->pool.size() < (size_t)(4 * P.p.m + 16)) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) break;
      prof->pool.push_back(e);
    }
  }
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    ctx->use_graphs = false;
    return enqueue_solve(P, ws, ctx->stream, rows, ctx->host_info, prof);
  }
  int rc = enqueue_solve(P, ws, ctx->stream, rows, ctx->host_info, prof);
  hipError_t e = hipStreamEndCapture(ctx->stream, &graph);
  hipGraphExec_t exec = nullptr;
  if (rc == FAB_OK && e == hipSuccess && graph) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (rc != FAB_OK || e != hipSuccess || !exec) {
    (void)hipGetLastError();
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    ctx->use_graphs = false;
    if (prof) { prof->marks.clear(); prof->used = 0; }
    return enqueue_solve(P, ws, ctx->stream, rows, ctx->host_info, prof);
  }
  fab_ctx_s::GraphEntry ge;
  ge.key = key;
  ge.graph = graph;
  ge.exec = exec;
  if (prof) {
    ge.marks = prof->marks;
    ge.events_used = prof->used;
  }
  ge.last_use = ++ctx->graph_clock;
  if (ctx->graphs.size() >= 8) {
    auto lru = std::min_element(ctx->graphs.begin(), ctx->graphs.end(),
                                [](const fab_ctx_s::GraphEntry& a, const fab_ctx_s::GraphEntry& b) {
                                  return a.last_use < b.last_use;
                                });
    hipGraphExecDestroy(lru->exec);
    hipGraphDestroy(lru->graph);
    ctx->graphs.erase(lru);
  }
  ctx->graphs.push_back(ge);
  return hipGraphLaunch(exec, ctx->stream) == hipSuccess ? FAB_OK : FAB_EDEVICE;
}

// ws_fixed != nullptr: the workspace (and the sampled SRHT rows behind it) is
// the caller-supplied region of fixed_bytes instead of a block of the arena,
// launched directly (no graph), nothing allocated.
static int solve_impl(fab_ctx ctx, fab_matrix A, const double* b, int nrhs, fab_func f, const fab_params* p,
                      double* out, fab_info* info, const fab_diag* diag, char* ws_fixed = nullptr,
                      size_t fixed_bytes = 0) {
  if (!ctx || !A || !b || !out || !p || A->ctx != ctx) return FAB_EINVAL;
  const double t0 = now_us();
  std::lock_guard<std::mutex> slk(ctx->solve_mu);
  hipSetDevice(ctx->device);
  int esize = esize_for(p->prec == FAB_PREC_FP64 ? FAB_PREC_FP64 : FAB_PREC_FP32);
  Plan P;
  std::vector<fab_info> fi;
  char* ws = nullptr;
  int rc = FAB_OK;
  bool fell_back = false;
  for (int attempt = 0; attempt < 2; ++attempt) {
    rc = make_plan(A, nrhs, f, p, esize, P);
    if (rc != FAB_OK) return rc;
    P.b = b;
    P.out = out;
    if (ws_fixed) {
      if (align256(P.bytes) + align256((size_t)P.p.s * 4) > fixed_bytes) return FAB_ESCRATCH;
      ws = ws_fixed;
    } else {
      std::unique_lock<std::mutex> lk(ctx->mu);
      if (!ctx->arena.could_ever_fit(P.bytes)) return FAB_ENOMEM;
      while (!(ws = (char*)ctx->arena.alloc(P.bytes))) {
        bool running = false;
        for (auto& kv : ctx->reqs)
          if (kv.second->state == 1) running = true;
        if (!running) return FAB_ENOMEM;
        ctx->cv.wait_for(lk, std::chrono::milliseconds(1));
      }
    }
    const int* rows = nullptr;
    if (P.p.sketch == FAB_SKETCH_SRHT) {
      if (ws_fixed) {
        int* r = (int*)(ws_fixed + align256(P.bytes));
        if (srht_sample_rows(r, 1LL << ilog2(A->n), P.p.s, sm64_out(P.p.seed, 2), ctx->stream) != hipSuccess)
          rc = FAB_EDEVICE;
        rows = r;
      } else {
        std::lock_guard<std::mutex> lk(ctx->mu);
        rows = srht_rows_cached(ctx, 1LL << ilog2(A->n), P.p.s, P.p.seed, ctx->stream, &rc);
      }
    }
    if (rc == FAB_OK)
      rc = ws_fixed ? enqueue_solve(P, ws, ctx->stream, rows, ctx->host_info, nullptr,
                                    ctx->host_flag)
                    : launch_solve(ctx, P, ws, rows, f);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess && rc == FAB_OK) rc = FAB_EDEVICE;
    if (ctx->prof.mask) ctx->prof.harvest();
    fi.clear();
    if (rc == FAB_OK || rc == FAB_ENUMERIC) {
      const int rc2 = collect_info(P, ctx->host_info, fi);
      if (rc == FAB_OK) rc = rc2;
    }
    if (attempt == 0 && (rc == RC_RERUN_FP64 || needs_fp64_rerun(P, rc, fi))) {
      // FAB_PREC_AUTO: recompute the whole request with an FP64 basis
      if (!ws_fixed) {
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->arena.release(ws);
      }
      ws = nullptr;
      esize = 8;
      fell_back = true;
      continue;
    }
    break;
  }
  if (needs_refine(P, rc, fi)) {
    rc = enqueue_refine(P, ws, ctx->stream, nullptr, ctx->host_info, ctx->host_flag);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess && rc == FAB_OK) rc = FAB_EDEVICE;
    if (rc == FAB_OK) rc = collect_info(P, ctx->host_info, fi);
  }
  if (fell_back)
    for (auto& x : fi) x.fell_back = 1;
  if (diag && (rc == FAB_OK || rc == FAB_ENUMERIC)) {
    const int m = P.p.m, s = P.p.s;
    for (int q = 0; q < nrhs; ++q) {
      const char* dq = ws + P.oDense + (size_t)q * P.dense_stride * 8;
      hipError_t e = hipSuccess;
      if (diag->hbar)
        e = hipMemcpy(diag->hbar + (size_t)q * (m + 1) * m, ws + P.oH + (size_t)q * (m + 1) * m * 8,
                      (size_t)(m + 1) * m * 8, hipMemcpyDeviceToHost);
      if (e == hipSuccess && diag->eta)
        e = hipMemcpy(diag->eta + (size_t)q * (m + 1), ws + P.oEta + (size_t)q * (m + 1) * 8, (size_t)(m + 1) * 8,
                      hipMemcpyDeviceToHost);
      if (e == hipSuccess && diag->y)
        e = hipMemcpy(diag->y + (size_t)q * m, dq + (P.oDVec + 2 * (size_t)m) * 8, (size_t)m * 8, hipMemcpyDeviceToHost);
      if (e == hipSuccess && diag->c)
        e = hipMemcpy(diag->c + (size_t)q * m, dq + P.oDVec * 8, (size_t)m * 8, hipMemcpyDeviceToHost);
      if (e == hipSuccess && diag->sv) {
        std::vector<double> raw((size_t)s * (m + 1)), eta(m + 1);
        e = hipMemcpy(raw.data(), ws + P.oS + (size_t)q * s * (m + 1) * 8, raw.size() * 8, hipMemcpyDeviceToHost);
        if (e == hipSuccess)
          e = hipMemcpy(eta.data(), ws + P.oEta + (size_t)q * (m + 1) * 8, (size_t)(m + 1) * 8, hipMemcpyDeviceToHost);
        for (int j = 0; j <= m && e == hipSuccess; ++j)
          for (int r = 0; r < s; ++r)
            diag->sv[(size_t)q * s * (m + 1) + (size_t)j * s + r] = eta[j] > 0 ? raw[(size_t)j * s + r] / eta[j] : 0.0;
      }
      if (e != hipSuccess) rc = FAB_EDEVICE;
    }
  }
  if (!ws_fixed) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->arena.release(ws);
  }
  const double t1 = now_us();
  if (info && !fi.empty())
    for (int q = 0; q < nrhs; ++q) {
      info[q] = fi[q];
      info[q].latency_us = t1 - t0;
    }
  return rc;
}

int fab_solve(fab_ctx ctx, fab_matrix A, const double* b, int nrhs, fab_func f, const fab_params* p, double* out,
              fab_info* info) {
  return solve_impl(ctx, A, b, nrhs, f, p, out, info, nullptr);
}

int fab_solve_diag(fab_ctx ctx, fab_matrix A, const double* b, int nrhs, fab_func f, const fab_params* p,
                   double* out, fab_info* info, const fab_diag* diag) {
  return solve_impl(ctx, A, b, nrhs, f, p, out, info, diag);
}


int fab_profile_enable(fab_ctx ctx, int class_mask) {
  if (!ctx || class_mask < 0 || class_mask >= (1 << FAB_K_NCLASS)) return FAB_EINVAL;
  std::lock_guard<std::mutex> slk(ctx->solve_mu);
  ctx->prof.mask = class_mask;
  return FAB_OK;
}

int fab_profile_read(fab_ctx ctx, int cls, long long* launches, double* total_ms, int reset) {
  if (!ctx || cls < 0 || cls >= FAB_K_NCLASS) return FAB_EINVAL;
  std::lock_guard<std::mutex> slk(ctx->solve_mu);
  if (launches) *launches = ctx->prof.count[cls];
  if (total_ms) *total_ms = ctx->prof.total_ms[cls];
  if (reset) {
    ctx->prof.count[cls] = 0;
    ctx->prof.total_ms[cls] = 0.0;
  }
  return FAB_OK;
}

int fab_submit(fab_ctx ctx, fab_matrix A, const double* b, int nrhs, fab_func f, const fab_params* p, double* out,
               fab_request* req) {
  if (!ctx || !A || !b || !out || !p || !req || A->ctx != ctx) return FAB_EINVAL;
  auto r = std::make_shared<Request>();
  int first_prec = p->prec == FAB_PREC_FP64 ? FAB_PREC_FP64 : FAB_PREC_FP32;
  int rc = make_plan(A, nrhs, f, p, esize_for(first_prec), r->plan);
  if (rc != FAB_OK) return rc;
  r->plan.b = b;
  r->plan.out = out;
  hipSetDevice(ctx->device);
  if (hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming) != hipSuccess) return FAB_EDEVICE;
  r->t_submit = now_us();
  std::lock_guard<std::mutex> lk(ctx->mu);
  if (!ctx->arena.could_ever_fit(r->plan.bytes)) {
    hipEventDestroy(r->done_ev);
    return FAB_ENOMEM;
  }
  r->host_info = (double*)ctx->pinned.get();
  if (r->host_info) r->flag_host = (int*)ctx->pinned.get();
  if (!r->host_info || !r->flag_host) {
    hipEventDestroy(r->done_ev);
    ctx->pinned.put(r->host_info);
    return FAB_EDEVICE;
  }
  r->id = ctx->next_id++;
  r->plan.A->refs.fetch_add(1);   // released at retirement
  ctx->reqs[r->id] = r;
  ctx->queue.push_back(r->id);
  *req = r->id;
  ctx->cv.notify_all();
  return FAB_OK;
}

int fab_hold(fab_ctx ctx, int hold) {
  if (!ctx) return FAB_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->hold = hold != 0;
  ctx->cv.notify_all();
  return FAB_OK;
}

int fab_set_block_limit(fab_ctx ctx, int max_rhs) {
  if (!ctx || max_rhs < 1 || max_rhs > 32) return FAB_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->block_max = max_rhs;
  return FAB_OK;
}

static int finish_request(fab_ctx ctx, std::unordered_map<uint64_t, std::shared_ptr<Request>>::iterator it,
                          fab_info* info) {
  Request& r = *it->second;
  const int rc = r.status;
  if (info)
    for (size_t q = 0; q < r.info.size(); ++q) info[q] = r.info[q];
  hipEventDestroy(r.done_ev);
  ctx->pinned.put(r.host_info);
  ctx->pinned.put(r.flag_host);
  ctx->reqs.erase(it);
  return rc;
}

int fab_poll(fab_ctx ctx, fab_request req, int* done, fab_info* info) {
  if (!ctx || !done) return FAB_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  auto it = ctx->reqs.find(req);
  if (it == ctx->reqs.end()) return FAB_ENOTFOUND;
  if (it->second->state != 2) { *done = 0; return FAB_OK; }
  *done = 1;
  return finish_request(ctx, it, info);
}

int fab_wait(fab_ctx ctx, fab_request req, fab_info* info) {
  if (!ctx) return FAB_EINVAL;
  std::unique_lock<std::mutex> lk(ctx->mu);
  auto it = ctx->reqs.find(req);
  if (it == ctx->reqs.end()) return FAB_ENOTFOUND;
  // hold the request itself across the wait: a submit from another thread
  // may rehash the table (invalidating iterators) while mu is released
  const std::shared_ptr<Request> r = it->second;
  ctx->cv.wait(lk, [&] { return r->state == 2; });
  it = ctx->reqs.find(req);
  if (it == ctx->reqs.end()) return FAB_ENOTFOUND;   // released by a concurrent fab_poll/fab_wait
  return finish_request(ctx, it, info);
}

int fab_finalize(fab_ctx ctx) {
  if (!ctx) return FAB_EINVAL;
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->stop = true;
    ctx->hold = false;
    ctx->cv.notify_all();
  }
  if (ctx->sched.joinable()) ctx->sched.join();
  hipSetDevice(ctx->device);
  for (auto& kv : ctx->reqs) {
    if (kv.second->worker.joinable()) kv.second->worker.join();
    if (kv.second->done_ev) hipEventDestroy(kv.second->done_ev);
  }
  ctx->reqs.clear();
  for (auto* M : ctx->matrices) delete M;
  ctx->matrices.clear();
  for (auto s : ctx->pool) {
    hipStreamSynchronize(s);
    hipStreamDestroy(s);
  }
  if (ctx->own_stream) hipStreamDestroy(ctx->stream);
  else hipStreamSynchronize(ctx->stream);
  for (auto& g : ctx->graphs) {
    hipGraphExecDestroy(g.exec);
    hipGraphDestroy(g.graph);
  }
  ctx->graphs.clear();
  ctx->pinned.release_all();
  if (ctx->host_info) hipHostFree(ctx->host_info);
  if (ctx->host_flag) hipHostFree(ctx->host_flag);
  for (auto ev : ctx->prof.pool) hipEventDestroy(ev);
  if (ctx->arena.owned) hipFree(ctx->arena.base);
  delete ctx;
  return FAB_OK;
}

}  // extern "C"

namespace fab {
// The blocking solve on a caller-supplied device workspace (the static
// scratch of fab_solve_noalloc, noalloc.hip).
int solve_fixed_workspace(fab_ctx ctx, fab_matrix A, const double* b, int nrhs, fab_func f, const fab_params* p,
                          double* out, fab_info* info, char* ws, size_t bytes) {
  if (!ws) return FAB_EINVAL;
  return solve_impl(ctx, A, b, nrhs, f, p, out, info, nullptr, ws, bytes);
}
int ctx_device(fab_ctx ctx) { return ctx ? ctx->device : -1; }
}  // namespace fab
