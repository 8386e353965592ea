// Optimization of the product basis (Sec. "Optimization of the MPB"): keep
// only the Coulomb eigenfunctions E_mu with eigenvalue v_mu >= v_min.  The
// basis here is the Coulomb eigenbasis (v diagonal), so the optimization
// compacts the rows of U and the entries of v, in their original order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "gw_internal.hpp"

namespace gw {
namespace {

// positions of the kept rows: exclusive prefix sum of (v >= v_min), one
// workgroup of 1024 lanes walking the rows in blocks.
__global__ __launch_bounds__(1024) void basis_scan_kernel(int N, const double* __restrict__ v, double v_min,
                                                          int n_keep, int* __restrict__ src_of_dst) {
  __shared__ int sums[1024];
  __shared__ int base;
  if (threadIdx.x == 0) base = 0;
  // slots the selection does not reach (device values disagreeing with the
  // count) stay -1 and are skipped by the gather
  for (int i = threadIdx.x; i < n_keep; i += 1024) src_of_dst[i] = -1;
  __syncthreads();
  for (int b0 = 0; b0 < N; b0 += 1024) {
    const int i = b0 + (int)threadIdx.x;
    const int keep = (i < N && v[i] >= v_min) ? 1 : 0;
    sums[threadIdx.x] = keep;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {     // inclusive Hillis-Steele scan
      const int add = threadIdx.x >= (unsigned)off ? sums[threadIdx.x - off] : 0;
      __syncthreads();
      sums[threadIdx.x] += add;
      __syncthreads();
    }
    const int pos = base + sums[threadIdx.x] - 1;
    if (keep && pos < n_keep) src_of_dst[pos] = i;
    __syncthreads();
    if (threadIdx.x == 1023) base += sums[1023];
    __syncthreads();
  }
}

// row gather: U_out[d][:] = U[src[d]][:], v_out[d] = v[src[d]] (16-byte
// vectors when the row length allows, else bytes).
__global__ void basis_gather_kernel(int n_keep, size_t row_bytes, const int* __restrict__ src,
                                    const unsigned char* __restrict__ U, const double* __restrict__ v,
                                    unsigned char* __restrict__ U_out, double* __restrict__ v_out) {
  for (int d = blockIdx.y; d < n_keep; d += gridDim.y) {
    const int s = src[d];
    if (s < 0) continue;
    if (blockIdx.x == 0 && threadIdx.x == 0) v_out[d] = v[s];
    const unsigned char* in = U + (size_t)s * row_bytes;
    unsigned char* out = U_out + (size_t)d * row_bytes;
    if (row_bytes % 16 == 0) {
      const size_t n = row_bytes / 16;
      for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        reinterpret_cast<uint4*>(out)[e] = reinterpret_cast<const uint4*>(in)[e];
    } else {
      for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < row_bytes;
           e += (size_t)gridDim.x * blockDim.x)
        out[e] = in[e];
    }
  }
}

}  // namespace
}  // namespace gw

using namespace gw;

extern "C" int gw_basis_select_count(int N, const double* v_host, double v_min, int* n_keep_host) {
  if (N < 1 || !v_host || !n_keep_host) return fail(GW_ERR_INVALID_ARG, "gw_basis_select_count: bad arguments");
  if (!std::isfinite(v_min)) return fail(GW_ERR_INVALID_ARG, "gw_basis_select_count: v_min must be finite");
  int n = 0;
  for (int i = 0; i < N; ++i) {
    if (!std::isfinite(v_host[i])) return fail(GW_ERR_INVALID_ARG, "gw_basis_select_count: non-finite v");
    n += v_host[i] >= v_min ? 1 : 0;
  }
  *n_keep_host = n;
  return GW_OK;
}

extern "C" int gw_basis_select(void* stream, int N, int R, int elem_bytes, const void* U, const double* v,
                               double v_min, int n_keep, void* U_out, double* v_out, int* src_of_dst) {
  if (N < 1 || R < 1 || (elem_bytes != 4 && elem_bytes != 8 && elem_bytes != 16))
    return fail(GW_ERR_INVALID_ARG, "gw_basis_select: N, R >= 1 and elem_bytes in {4, 8, 16}");
  if (n_keep < 0 || n_keep > N) return fail(GW_ERR_INVALID_ARG, "gw_basis_select: n_keep out of range");
  if (!std::isfinite(v_min)) return fail(GW_ERR_INVALID_ARG, "gw_basis_select: v_min must be finite");
  if (!U || !v) return fail(GW_ERR_INVALID_ARG, "gw_basis_select: NULL pointer");
  if (n_keep == 0) return GW_OK;   // nothing kept: the outputs are not touched (and may be NULL)
  if (!U_out || !v_out || !src_of_dst) return fail(GW_ERR_INVALID_ARG, "gw_basis_select: NULL pointer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(basis_scan_kernel, dim3(1), dim3(1024), 0, s, N, v, v_min, n_keep, src_of_dst);
  GW_LAUNCHED("basis_scan_kernel");
  const size_t row_bytes = (size_t)R * elem_bytes;
  const unsigned gx = (unsigned)std::min<size_t>(64, (row_bytes / 16 + 255) / 256 + 1);
  hipLaunchKernelGGL(basis_gather_kernel, dim3(gx, std::min(n_keep, 65535)), dim3(256), 0, s, n_keep, row_bytes,
                     src_of_dst,
                     static_cast<const unsigned char*>(U), v, static_cast<unsigned char*>(U_out), v_out);
  GW_LAUNCHED("basis_gather_kernel");
  return GW_OK;
}
