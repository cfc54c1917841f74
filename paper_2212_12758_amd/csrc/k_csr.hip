// Operator products that run as launches of their own:
//
//  * y = A x for the CSR operator (the operator application of every Krylov
//    step, Algorithm 2 and Algorithm 1, when A is given as a sparse matrix);
//  * y = A (A x) for the sign function, sign(A) b = (A^2)^{-1/2} (A b)
//    (Section 5.1.3): the basis is built for A^2, which is applied as two
//    products with A (stencil or CSR), the intermediate A x kept in FP64, so
//    A^2 is never formed;
//  * y = A x of FP64 vectors (the start vector A b of the sign function).
//
// CSR scheme:
//
// x and y are [n][nrhs] (element (row r, rhs q) at r*nrhs + q); x is FP32 or
// FP64 (a basis column or an FP64 vector), y is FP64 (the w~ buffer read by
// the passes that follow).  The nonzeros of a block of rows are consecutive
// in memory, so a workgroup reads them as one coalesced stream instead of one
// row per thread:
//
//   * a workgroup owns 256 consecutive elements (256/nrhs rows);
//   * its nonzeros are taken in chunks of 4096 products: every thread loads
//     16 (col, val) pairs (with one rhs as 4 groups of 4 consecutive pairs in
//     16-byte loads, else one pair at a time at stride 256; all loads in
//     flight), then the 16 gathered x values, and writes the products val * x
//     to LDS;
//   * the thread of element (r, q) then adds the products of row r that fall
//     in the chunk, in increasing nonzero order.
//
// Every y element is the sum of its row's products in nonzero order (chunks
// are visited in order), so the result is independent of the launch and
// bitwise reproducible.  A row of any length is handled: it simply spans
// several chunks.
//
// Blocks are dispatched round-robin over the 8 XCDs; the logical row block of
// physical block b is remapped so that each XCD walks one contiguous eighth
// of the rows, keeping the x neighbourhoods of a locality-ordered matrix in
// that XCD's L2.
#include "k_basis.h"

namespace fab {

namespace {

constexpr int SPMV_BLOCK = 256;
constexpr int SPMV_PER_THREAD = 16;
constexpr int SPMV_CHUNK = SPMV_BLOCK * SPMV_PER_THREAD;   // products per chunk
constexpr int NXCD = 8;

template <typename T>
__global__ void __launch_bounds__(SPMV_BLOCK)
k_csr_spmv(const int* __restrict__ rowptr, const int* __restrict__ col, const float* __restrict__ val,
           const T* __restrict__ x, double* __restrict__ y, int n, int lognr) {
  __shared__ double prod[SPMV_CHUNK];
  const int nr = 1 << lognr;
  const int tid = threadIdx.x;
  const int G = gridDim.x, b = blockIdx.x;
  const int lb = (G % NXCD == 0) ? (b % NXCD) * (G / NXCD) + b / NXCD : b;
  const int rpb = SPMV_BLOCK >> lognr;                     // rows per block
  const int r0 = lb * rpb;
  const int r1 = r0 + rpb < n ? r0 + rpb : n;
  const int r = r0 + (tid >> lognr), q = tid & (nr - 1);
  const bool own = r < r1;
  const int pb = rowptr[r0], pe = rowptr[r1];
  const int a0 = own ? rowptr[r] : 0, a1 = own ? rowptr[r + 1] : 0;
  const int cpe = SPMV_CHUNK >> lognr;                     // nonzeros per chunk
  double acc = 0.0;
  for (int c0 = pb; c0 < pe; c0 += cpe) {
    const int ce = pe - c0 < cpe ? pe - c0 : cpe;          // nonzeros in this chunk
    const int cn = ce << lognr;                            // products in this chunk
    int cl[SPMV_PER_THREAD];
    float vl[SPMV_PER_THREAD];
#pragma unroll
    for (int k = 0; k < SPMV_PER_THREAD; ++k) {
      const int g = tid + k * SPMV_BLOCK;
      const int p = c0 + (g >> lognr);
      cl[k] = g < cn ? col[p] : 0;
      vl[k] = g < cn ? val[p] : 0.0f;
    }
    // g & (nr - 1) == q for every k: the block stride is a multiple of nrhs
#pragma unroll
    for (int k = 0; k < SPMV_PER_THREAD; ++k) {
      const int g = tid + k * SPMV_BLOCK;
      const double xv = g < cn ? (double)x[((long long)cl[k] << lognr) + q] : 0.0;
      prod[g] = (double)vl[k] * xv;
    }
    __syncthreads();
    const int lo = a0 > c0 ? a0 : c0;
    const int hi = a1 < c0 + ce ? a1 : c0 + ce;
    for (int p = lo; p < hi; ++p) acc += prod[((p - c0) << lognr) + q];
    __syncthreads();
  }
  if (own) y[((long long)r << lognr) + q] = acc;
}

// One right-hand side: the same scheme with 16-byte loads.  Chunks start on
// a multiple of 4 nonzeros (the index and value arrays start on 256-byte
// boundaries), each thread loads 4 groups of 4 consecutive (col, val) pairs,
// and the up to 3 nonzeros of the previous row block that precede the first
// row are loaded but never summed.
template <typename T>
__global__ void __launch_bounds__(SPMV_BLOCK)
k_csr_spmv1(const int* __restrict__ rowptr, const int* __restrict__ col, const float* __restrict__ val,
            const T* __restrict__ x, double* __restrict__ y, int n) {
  constexpr int NV = SPMV_PER_THREAD / 4;
  __shared__ double prod[SPMV_CHUNK];
  const int tid = threadIdx.x;
  const int G = gridDim.x, b = blockIdx.x;
  const int lb = (G % NXCD == 0) ? (b % NXCD) * (G / NXCD) + b / NXCD : b;
  const int r0 = lb * SPMV_BLOCK;
  const int r1 = r0 + SPMV_BLOCK < n ? r0 + SPMV_BLOCK : n;
  const int r = r0 + tid;
  const bool own = r < r1;
  const int pb = rowptr[r0], pe = rowptr[r1];
  const int a0 = own ? rowptr[r] : 0, a1 = own ? rowptr[r + 1] : 0;
  double acc = 0.0;
  for (int c0 = pb & ~3; c0 < pe; c0 += SPMV_CHUNK) {
    int cl[SPMV_PER_THREAD];
    float vl[SPMV_PER_THREAD];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int q = c0 + 4 * (tid + v * SPMV_BLOCK);
      if (q + 4 <= pe) {
        const int4 c4 = *reinterpret_cast<const int4*>(col + q);
        const float4 v4 = *reinterpret_cast<const float4*>(val + q);
        cl[4 * v] = c4.x;
        cl[4 * v + 1] = c4.y;
        cl[4 * v + 2] = c4.z;
        cl[4 * v + 3] = c4.w;
        vl[4 * v] = v4.x;
        vl[4 * v + 1] = v4.y;
        vl[4 * v + 2] = v4.z;
        vl[4 * v + 3] = v4.w;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          cl[4 * v + j] = q + j < pe ? col[q + j] : 0;
          vl[4 * v + j] = q + j < pe ? val[q + j] : 0.0f;
        }
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        prod[4 * (tid + v * SPMV_BLOCK) + j] = (double)vl[4 * v + j] * (double)x[cl[4 * v + j]];
    __syncthreads();
    const int lo = a0 > c0 ? a0 : c0;
    const int hi = a1 < c0 + SPMV_CHUNK ? a1 : c0 + SPMV_CHUNK;
    for (int p = lo; p < hi; ++p) acc += prod[p - c0];
    __syncthreads();
  }
  if (own) y[r] = acc;
}

// y = A x for the stencil operator, x FP32 or FP64 [n][nrhs], y FP64.
template <typename T>
__global__ void __launch_bounds__(256) k_stencil_apply(SolveDev d, const T* __restrict__ x, double* __restrict__ y) {
  const long long nel = (long long)d.n * d.nrhs;
  for (long long e = ((long long)blockIdx.x * 256 + threadIdx.x) * EPT; e < nel;
       e += (long long)gridDim.x * 256 * EPT) {
    double c[EPT], w[EPT];
    get8(x, e, nel, c);
    stencil8(d, x, e, nel, c, w);
    if (e + EPT <= nel) {
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        double2 o;
        o.x = w[2 * h];
        o.y = w[2 * h + 1];
        *reinterpret_cast<double2*>(y + e + 2 * h) = o;
      }
    } else {
      for (int j = 0; j < EPT; ++j)
        if (e + j < nel) y[e + j] = w[j];
    }
  }
}

hipError_t stencil_apply(const SolveDev& d, const void* x, int esize, double* y, hipStream_t st) {
  const long long nel = (long long)d.n * d.nrhs;
  long long g = (nel + 256 * EPT - 1) / (256 * EPT);
  if (g > 4096) g = 4096;
  if (g == 0) return hipSuccess;
  if (esize == 4)
    hipLaunchKernelGGL(k_stencil_apply<float>, dim3((unsigned)g), dim3(256), 0, st, d, (const float*)x, y);
  else
    hipLaunchKernelGGL(k_stencil_apply<double>, dim3((unsigned)g), dim3(256), 0, st, d, (const double*)x, y);
  return hipGetLastError();
}

}  // namespace

hipError_t csr_spmv(const SolveDev& d, const void* x, int esize, double* y, hipStream_t st) {
  const int rpb = SPMV_BLOCK >> d.lognrhs;
  const long long g = ((long long)d.n + rpb - 1) / rpb;
  if (g > 0x7fffffffLL) return hipErrorInvalidValue;
  if (g == 0) return hipSuccess;
  if (d.nrhs == 1) {
    if (esize == 4)
      hipLaunchKernelGGL(k_csr_spmv1<float>, dim3((unsigned)g), dim3(SPMV_BLOCK), 0, st, d.rowptr, d.col, d.val,
                         (const float*)x, y, d.n);
    else
      hipLaunchKernelGGL(k_csr_spmv1<double>, dim3((unsigned)g), dim3(SPMV_BLOCK), 0, st, d.rowptr, d.col, d.val,
                         (const double*)x, y, d.n);
    return hipGetLastError();
  }
  if (esize == 4)
    hipLaunchKernelGGL(k_csr_spmv<float>, dim3((unsigned)g), dim3(SPMV_BLOCK), 0, st, d.rowptr, d.col, d.val,
                       (const float*)x, y, d.n, d.lognrhs);
  else
    hipLaunchKernelGGL(k_csr_spmv<double>, dim3((unsigned)g), dim3(SPMV_BLOCK), 0, st, d.rowptr, d.col, d.val,
                       (const double*)x, y, d.n, d.lognrhs);
  return hipGetLastError();
}

hipError_t operator_product(const SolveDev& d, const void* x, int esize, double* y, hipStream_t st) {
  switch (d.prod) {
    case PROD_CSR:
      return csr_spmv(d, x, esize, y, st);
    case PROD_SQ_STENCIL: {
      const hipError_t r = stencil_apply(d, x, esize, d.wtmp, st);
      return r != hipSuccess ? r : stencil_apply(d, d.wtmp, 8, y, st);
    }
    case PROD_SQ_CSR: {
      const hipError_t r = csr_spmv(d, x, esize, d.wtmp, st);
      return r != hipSuccess ? r : csr_spmv(d, d.wtmp, 8, y, st);
    }
    default:
      return hipErrorInvalidValue;
  }
}

// y = A x for FP64 x with the operator A itself (stencil or CSR), whatever
// the basis is built for: the start vector A b of the sign function.
hipError_t apply_operator(const SolveDev& d, const double* x, double* y, hipStream_t st) {
  if (d.prod == PROD_CSR || d.prod == PROD_SQ_CSR) return csr_spmv(d, x, 8, y, st);
  return stencil_apply(d, x, 8, y, st);
}

}  // namespace fab
