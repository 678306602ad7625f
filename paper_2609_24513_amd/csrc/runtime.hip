// Error reporting, version and small blob queries of the C ABI.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>

#include "common.h"

namespace pr {

namespace {
thread_local char g_err[512] = "";

__global__ void k_boxes(const void* blob, int64_t n, float* boxes) {
  const BlobHeader* h = reinterpret_cast<const BlobHeader*>(blob);
  const MeshDesc* md = reinterpret_cast<const MeshDesc*>(reinterpret_cast<const char*>(blob) + h->off_mesh);
  int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; m < n; m += (int64_t)gridDim.x * blockDim.x)
    for (int k = 0; k < 6; ++k) boxes[6 * m + k] = md[m].box[k];
}

__global__ void k_exponents(const void* blob, int32_t* out) {
  const BlobHeader* h = reinterpret_cast<const BlobHeader*>(blob);
  out[0] = h->exp_lo;
  out[1] = h->exp_hi;
}

__global__ void k_edges(const void* blob, int64_t n, int32_t* counts) {
  const BlobHeader* h = reinterpret_cast<const BlobHeader*>(blob);
  const MeshDesc* md = reinterpret_cast<const MeshDesc*>(reinterpret_cast<const char*>(blob) + h->off_mesh);
  int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (; m < n; m += (int64_t)gridDim.x * blockDim.x) counts[m] = md[m].n_edges;
}
}  // namespace

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

int hip_fail(hipError_t e, const char* what) {
  set_error("%s: %s", what, hipGetErrorString(e));
  return PR_E_DEVICE;
}

}  // namespace pr

extern "C" const char* pr_last_error(void) { return pr::g_err; }

extern "C" int pr_abi_version(void) { return PR_ABI_VERSION; }

extern "C" int blob_mesh_boxes(const void* blob, int64_t n_meshes, float* boxes, void* stream) {
  if (!blob || n_meshes < 0 || (n_meshes > 0 && !boxes)) { pr::set_error("bad argument"); return PR_E_ARG; }
  if (n_meshes == 0) return PR_OK;
  hipLaunchKernelGGL(pr::k_boxes, dim3(pr::grid_for(n_meshes, 256)), dim3(256), 0, (hipStream_t)stream, blob,
                     n_meshes, boxes);
  PR_HIP(hipGetLastError());
  return PR_OK;
}

extern "C" int blob_edge_counts(const void* blob, int64_t n_meshes, int32_t* counts, void* stream) {
  if (!blob || n_meshes < 0 || (n_meshes > 0 && !counts)) { pr::set_error("bad argument"); return PR_E_ARG; }
  if (n_meshes == 0) return PR_OK;
  hipLaunchKernelGGL(pr::k_edges, dim3(pr::grid_for(n_meshes, 256)), dim3(256), 0, (hipStream_t)stream, blob,
                     n_meshes, counts);
  PR_HIP(hipGetLastError());
  return PR_OK;
}

extern "C" int blob_coord_exponents(const void* blob, int32_t* exps, void* stream) {
  if (!blob || !exps) { pr::set_error("bad argument"); return PR_E_ARG; }
  hipLaunchKernelGGL(pr::k_exponents, dim3(1), dim3(1), 0, (hipStream_t)stream, blob, exps);
  PR_HIP(hipGetLastError());
  return PR_OK;
}
