// k_misc.hip -- direct summation (Eq. 1) and the leapfrog kick / drift.
#include "nbody_internal.h"

namespace nb {

// Eq. 1 by direct summation, FP32: each lane owns one i, j-tiles of 256 are
// staged in LDS and read by broadcast. Same interaction arithmetic as the
// walk's flush, so it calibrates the walk's arithmetic rate. The j == i term
// contributes exactly zero because eps > 0.
__global__ __launch_bounds__(256) void k_direct(int64_t n, const float *__restrict__ x,
                                                const float *__restrict__ y,
                                                const float *__restrict__ z,
                                                const float *__restrict__ m, float G,
                                                float eps2, float *__restrict__ ax,
                                                float *__restrict__ ay,
                                                float *__restrict__ az) {
  __shared__ float4 tile[256];
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
  if (i < n) pi = make_float4(x[i], y[i], z[i], m[i]);
  float sx = 0.f, sy = 0.f, sz = 0.f;
  for (int64_t j0 = 0; j0 < n; j0 += 256) {
    const int64_t j = j0 + threadIdx.x;
    tile[threadIdx.x] = j < n ? make_float4(x[j], y[j], z[j], m[j]) : make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    const int cnt = (int)min((int64_t)256, n - j0);
#pragma unroll 8
    for (int k = 0; k < cnt; ++k) {
      const float4 e = tile[k];
      const float dx = e.x - pi.x, dy = e.y - pi.y, dz = e.z - pi.z;
      const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
      const float rinv = __builtin_amdgcn_rsqf(r2);
      const float mr = e.w * rinv;
      const float f = mr * (rinv * rinv);
      sx = __builtin_fmaf(f, dx, sx);
      sy = __builtin_fmaf(f, dy, sy);
      sz = __builtin_fmaf(f, dz, sz);
    }
    __syncthreads();
  }
  if (i < n) {
    ax[i] = G * sx;
    ay[i] = G * sy;
    az[i] = G * sz;
  }
}

// v += a * (dt/2), FP32, one rounding per operation.
__global__ __launch_bounds__(256) void k_kick(int64_t n, float *__restrict__ vx,
                                              float *__restrict__ vy, float *__restrict__ vz,
                                              const float *__restrict__ ax,
                                              const float *__restrict__ ay,
                                              const float *__restrict__ az, float hdt) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float kx = ax[i] * hdt, ky = ay[i] * hdt, kz = az[i] * hdt;
    vx[i] = vx[i] + kx;
    vy[i] = vy[i] + ky;
    vz[i] = vz[i] + kz;
  }
}

// x += v * dt in FP64 and the FP32 image of x for the tree.
__global__ __launch_bounds__(256) void k_drift(int64_t n, double *__restrict__ x,
                                               double *__restrict__ y,
                                               double *__restrict__ z,
                                               const float *__restrict__ vx,
                                               const float *__restrict__ vy,
                                               const float *__restrict__ vz, double dt,
                                               float *__restrict__ x32, SortedOut so) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double dx = (double)vx[i] * dt, dy = (double)vy[i] * dt, dz = (double)vz[i] * dt;
    const double nx = x[i] + dx, ny = y[i] + dy, nz = z[i] + dz;
    x[i] = nx;
    y[i] = ny;
    z[i] = nz;
    store_position(i, n, (float)nx, (float)ny, (float)nz, x32, so);
  }
}

static int grid_1d(int64_t n) {
  int64_t g = cdiv(n, 256 * 4);
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

void launch_direct(int64_t n, const float *x, const float *y, const float *z,
                   const float *m, float G, float eps, float *ax, float *ay, float *az,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_direct, dim3(cdiv(n, 256)), dim3(256), 0, st, n, x, y, z, m, G,
                     eps * eps, ax, ay, az);
}

void launch_kick(int64_t n, float *vx, float *vy, float *vz, const float *ax,
                 const float *ay, const float *az, float hdt, hipStream_t st) {
  hipLaunchKernelGGL(k_kick, dim3(grid_1d(n)), dim3(256), 0, st, n, vx, vy, vz, ax, ay, az,
                     hdt);
}

void launch_drift(int64_t n, double *x, double *y, double *z, const float *vx,
                  const float *vy, const float *vz, double dt, float *x32, SortedOut so,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_drift, dim3(grid_1d(n)), dim3(256), 0, st, n, x, y, z, vx, vy, vz,
                     dt, x32, so);
}


// asort[s] = (a, |a|) of caller index perm[s]; |a| rounded as in the MAC.
__global__ __launch_bounds__(256) void k_asort_gather(const uint32_t *__restrict__ perm,
                                                      int64_t n, const float *__restrict__ ax,
                                                      const float *__restrict__ ay,
                                                      const float *__restrict__ az,
                                                      float4 *__restrict__ asort) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t o = perm[s];
    const float x = ax[o], y = ay[o], z = az[o];
    asort[s] = make_float4(x, y, z, sqrt_rn(__builtin_fmaf(z, z, __builtin_fmaf(y, y, x * x))));
  }
}

void launch_asort_gather(const uint32_t *perm, int64_t n, const float *ax, const float *ay,
                         const float *az, float4 *asort, hipStream_t st) {
  int64_t g = cdiv(n, 256 * 4);
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_asort_gather, dim3(g), dim3(256), 0, st, perm, n, ax, ay, az, asort);
}

// After a rebuild: the mirror in the new key order from the mirror in the
// old one, tmp[s] = asort[inv_old[perm_new[s]]], then copied back. Particles
// move little between builds, so the reads of the old mirror are nearly in
// order (one random 4-byte read of inv_old instead of three of a_old).
__global__ __launch_bounds__(256) void k_asort_remap(const uint32_t *__restrict__ perm,
                                                     const uint32_t *__restrict__ inv_old,
                                                     int64_t n, const float4 *__restrict__ asort,
                                                     float4 *__restrict__ tmp) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x)
    tmp[s] = asort[inv_old[perm[s]]];
}

__global__ __launch_bounds__(256) void k_copy_f4(const float4 *__restrict__ src, int64_t n,
                                                 float4 *__restrict__ dst) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x)
    dst[s] = src[s];
}

void launch_asort_remap(const uint32_t *perm, const uint32_t *inv_old, int64_t n,
                        float4 *asort, float4 *tmp, hipStream_t st) {
  int64_t g = cdiv(n, 256 * 4);
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_asort_remap, dim3(g), dim3(256), 0, st, perm, inv_old, n, asort, tmp);
  hipLaunchKernelGGL(k_copy_f4, dim3(g), dim3(256), 0, st, tmp, n, asort);
}

}  // namespace nb
