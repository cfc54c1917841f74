// Dispatch of the streaming basis kernels (the kernel templates are in
// k_basis.h, their variants are compiled per storage type and operator in
// k_basis_<type>_<op>.hip), the closing step, the combination V c and small
// utility kernels.
#include "k_basis.h"

namespace fab {

hipError_t basis_part_dots_f32_stencil(const SolveDev& d, int i, hipStream_t st, int nstream, int grid);
hipError_t basis_part_update_f32_stencil(const SolveDev& d, int i, hipStream_t st, size_t lds);
hipError_t basis_part_attributes_f32_stencil();
hipError_t basis_part_start_f32_stencil(const SolveDev& d, hipStream_t st, size_t lds);
hipError_t basis_part_dots_f32_csr(const SolveDev& d, int i, hipStream_t st, int nstream, int grid);
hipError_t basis_part_update_f32_csr(const SolveDev& d, int i, hipStream_t st, size_t lds);
hipError_t basis_part_attributes_f32_csr();
hipError_t basis_part_dots_f64_stencil(const SolveDev& d, int i, hipStream_t st, int nstream, int grid);
hipError_t basis_part_update_f64_stencil(const SolveDev& d, int i, hipStream_t st, size_t lds);
hipError_t basis_part_attributes_f64_stencil();
hipError_t basis_part_start_f64_stencil(const SolveDev& d, hipStream_t st, size_t lds);
hipError_t basis_part_dots_f64_csr(const SolveDev& d, int i, hipStream_t st, int nstream, int grid);
hipError_t basis_part_update_f64_csr(const SolveDev& d, int i, hipStream_t st, size_t lds);
hipError_t basis_part_attributes_f64_csr();

hipError_t basis_set_attributes() {
  hipError_t e = hipSuccess, r;
  if ((r = basis_part_attributes_f32_stencil()) != hipSuccess) e = r;
  if ((r = basis_part_attributes_f32_csr()) != hipSuccess) e = r;
  if ((r = basis_part_attributes_f64_stencil()) != hipSuccess) e = r;
  if ((r = basis_part_attributes_f64_csr()) != hipSuccess) e = r;
  return e;
}

hipError_t basis_start(const SolveDev& d, int esize, hipStream_t st, size_t lds) {
  return esize == 4 ? basis_part_start_f32_stencil(d, st, lds) : basis_part_start_f64_stencil(d, st, lds);
}
hipError_t basis_dots(const SolveDev& d, int esize, int i, hipStream_t st) {
  const bool csr = d.op == OP_CSR;
  if (esize == 4)
    return csr ? basis_part_dots_f32_csr(d, i, st, d.nblk, d.nblk) : basis_part_dots_f32_stencil(d, i, st, d.nblk, d.nblk);
  return csr ? basis_part_dots_f64_csr(d, i, st, d.nblk, d.nblk) : basis_part_dots_f64_stencil(d, i, st, d.nblk, d.nblk);
}
hipError_t basis_update(const SolveDev& d, int esize, int i, hipStream_t st, size_t lds) {
  const bool csr = d.op == OP_CSR;
  if (esize == 4) return csr ? basis_part_update_f32_csr(d, i, st, lds) : basis_part_update_f32_stencil(d, i, st, lds);
  return csr ? basis_part_update_f64_csr(d, i, st, lds) : basis_part_update_f64_stencil(d, i, st, lds);
}
hipError_t basis_finish(const SolveDev& d, int esize, hipStream_t st) {
  (void)esize;
  if (d.log_tile == 11) hipLaunchKernelGGL(k_finish<11>, dim3(d.nred), dim3(256), 0, st, d);
  else hipLaunchKernelGGL(k_finish<9>, dim3(d.nred), dim3(64), 0, st, d);
  return hipGetLastError();
}
hipError_t basis_combine(const SolveDev& d, int esize, const double* cf, int mmax, double* out, hipStream_t st) {
  const long long nel = (long long)d.n * d.nrhs;
  long long g = (nel + 256 * EPT - 1) / (256 * EPT);
  if (g > 4096) g = 4096;
  const bool nr1 = d.nrhs == 1;
  if (esize == 4) {
    if (nr1) hipLaunchKernelGGL((k_combine<float, true>), dim3((unsigned)g), dim3(256), 0, st, d, cf, mmax, out);
    else hipLaunchKernelGGL((k_combine<float, false>), dim3((unsigned)g), dim3(256), 0, st, d, cf, mmax, out);
  } else {
    if (nr1) hipLaunchKernelGGL((k_combine<double, true>), dim3((unsigned)g), dim3(256), 0, st, d, cf, mmax, out);
    else hipLaunchKernelGGL((k_combine<double, false>), dim3((unsigned)g), dim3(256), 0, st, d, cf, mmax, out);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ small utility kernels
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

// Blocked requests: the b vectors of g single-rhs requests into one
// interleaved [n][g] block (element (r, q) at r g + q), and the block's result
// back into each request's out.  g is a power of two <= 32.
__global__ void k_gather_cols(ColPtrs src, int logg, long long n, double* __restrict__ dst) {
  const long long tot = n << logg;
  const int gm = (1 << logg) - 1;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < tot; e += (long long)gridDim.x * 256)
    dst[e] = src.p[(int)(e & gm)][e >> logg];
}
__global__ void k_scatter_cols(const double* __restrict__ src, int logg, long long n, OutPtrs dst) {
  const long long tot = n << logg;
  const int gm = (1 << logg) - 1;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < tot; e += (long long)gridDim.x * 256)
    dst.p[(int)(e & gm)][e >> logg] = src[e];
}
static unsigned col_grid(long long tot) {
  long long g = (tot + 255) / 256;
  return (unsigned)(g > 4096 ? 4096 : (g < 1 ? 1 : g));
}
hipError_t gather_cols(const ColPtrs& src, int logg, long long n, double* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_cols, dim3(col_grid(n << logg)), dim3(256), 0, st, src, logg, n, dst);
  return hipGetLastError();
}
hipError_t scatter_cols(const double* src, int logg, long long n, const OutPtrs& dst, hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_cols, dim3(col_grid(n << logg)), dim3(256), 0, st, src, logg, n, dst);
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

