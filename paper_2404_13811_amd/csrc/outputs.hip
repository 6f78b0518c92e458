// Outputs of the MRCM-OS solve: cell pressures (zero mean when no side
// carries a pressure condition) and outward normal velocities on every face
// of every cell, with skeleton faces carrying the owning subdomain's value.
#include "local_common.h"

namespace mrcm {
namespace {

constexpr int RED = 256;

// Deterministic two-pass mean: fixed partition into npart blocks, fixed tree.
__device__ __forceinline__ void partial_sum(const double* __restrict__ p, int n, int b, int npart,
                                            double* __restrict__ partial) {
  __shared__ double s[RED];
  double acc = 0.0;
  for (int i = b * RED + threadIdx.x; i < n; i += npart * RED) acc += p[i];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int off = RED / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[b] = s[0];
}

__global__ void k_partial_sum(const double* __restrict__ p, int n, double* __restrict__ partial) {
  partial_sum(p, n, blockIdx.x, gridDim.x, partial);
}

__global__ void k_shift_copy(const double* __restrict__ p, int n, const double* __restrict__ partial,
                             int npart, int shift, double* __restrict__ out) {
  __shared__ double mean;
  if (threadIdx.x == 0) {
    double acc = 0.0;
    if (shift)
      for (int k = 0; k < npart; ++k) acc += partial[k];
    mean = acc / n;
  }
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = p[i] - mean;
}

__device__ __forceinline__ void flux_out(const Geo& g, const double* __restrict__ K,
                                         const double* __restrict__ p,
                                         const double* __restrict__ gflux,
                                         const double* __restrict__ bcv, double* __restrict__ out,
                                         int b) {
  const int ci = b * blockDim.x + threadIdx.x;
  if (ci >= g.ncells) return;
  int c[3], own[3];
  const int sub = cell_owner(g, ci, c, own);
  for (int a = 0; a < g.d; ++a)
    for (int s = 0; s < 2; ++s)
      out[(long long)ci * (2 * g.d) + 2 * a + s] = state_face_u(g, K, p, gflux, bcv, c, ci, own, sub, a, s);
}

__global__ void k_flux_out(Geo g, const double* __restrict__ K, const double* __restrict__ p,
                           const double* __restrict__ gflux, const double* __restrict__ bcv,
                           double* __restrict__ out) {
  flux_out(g, K, p, gflux, bcv, out, blockIdx.x);
}

// Flux output and the partial sums of the pressure mean in one launch:
// workgroups [0, npart) the sums (npart = 0: no mean), the rest the fluxes.
__global__ void k_flux_partial(Geo g, const double* __restrict__ K, const double* __restrict__ p,
                               const double* __restrict__ gflux, const double* __restrict__ bcv,
                               double* __restrict__ out, int npart, double* __restrict__ partial) {
  const int b = blockIdx.x;
  if (b < npart) partial_sum(p, g.ncells, b, npart, partial);
  else flux_out(g, K, p, gflux, bcv, out, b - npart);
}

}  // namespace

hipError_t launch_pressure_out(const Geo& g, const double* p, double* out, double* partial,
                               hipStream_t s) {
  const int n = g.ncells;
  const int npart = 64;
  if (g.neumann)
    hipLaunchKernelGGL(k_partial_sum, dim3(npart), dim3(RED), 0, s, p, n, partial);
  hipLaunchKernelGGL(k_shift_copy, dim3((n + 255) / 256), dim3(256), 0, s, p, n, partial, npart,
                     g.neumann, out);
  return hipGetLastError();
}

hipError_t launch_solution_out(const Geo& g, const double* K, const double* p, const double* gflux,
                               const double* bcv, double* p_out, double* flux_out, double* partial,
                               hipStream_t s) {
  const int n = g.ncells;
  const int npart = g.neumann ? 64 : 0;
  hipLaunchKernelGGL(k_flux_partial, dim3(npart + (n + 255) / 256), dim3(256), 0, s, g, K, p, gflux,
                     bcv, flux_out, npart, partial);
  hipLaunchKernelGGL(k_shift_copy, dim3((n + 255) / 256), dim3(256), 0, s, p, n, partial, 64,
                     g.neumann, p_out);
  return hipGetLastError();
}

hipError_t launch_flux_out(const Geo& g, const double* K, const double* p, const double* gflux,
                           const double* bcv, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_flux_out, dim3((g.ncells + 255) / 256), dim3(256), 0, s, g, K, p, gflux, bcv,
                     out);
  return hipGetLastError();
}

}  // namespace mrcm
