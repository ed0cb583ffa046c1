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

// Eq. 1 in FP64 for a subset of targets (the accuracy reference of the tree
// walk): inputs are FP32 positions and masses promoted to FP64; every pair
// j != i (by index) adds G m_j dx / (r^2 + eps^2)^(3/2) to a_i, G m_j |dx| /
// (r^2 + eps^2)^(3/2) to the scale A_i and -G m_j / (r^2 + eps^2)^(1/2) to
// phi_i. A workgroup takes 32 targets; its 8 lane groups ("phases") take
// every 8th particle of each 256-particle tile staged in LDS, and the 8
// partial sums of a target are added in phase order at the end.
constexpr int kD64Targets = 32;
constexpr int kD64Phases = 8;
__global__ __launch_bounds__(256) void k_direct64(int64_t n, const float *__restrict__ x,
                                                  const float *__restrict__ y,
                                                  const float *__restrict__ z,
                                                  const float *__restrict__ m, int64_t nt,
                                                  const int64_t *__restrict__ tgt, double G,
                                                  double eps2, double *__restrict__ ax,
                                                  double *__restrict__ ay,
                                                  double *__restrict__ az,
                                                  double *__restrict__ aabs,
                                                  double *__restrict__ phi) {
  __shared__ float4 tile[256];
  __shared__ double part[5][kD64Phases][kD64Targets];
  const int t = threadIdx.x % kD64Targets, ph = threadIdx.x / kD64Targets;
  const int64_t k = (int64_t)blockIdx.x * kD64Targets + t;
  const bool ok = k < nt;
  int64_t i = ok ? tgt[k] : -1;
  if (i >= n) i = -1;
  const bool live = i >= 0;  // a target outside [0, n) sums nothing
  const int64_t ii = live ? i : 0;
  const double xi = x[ii], yi = y[ii], zi = z[ii];
  double sx = 0.0, sy = 0.0, sz = 0.0, sa = 0.0, sp = 0.0;
  for (int64_t j0 = 0; j0 < n; j0 += 256) {
    const int64_t jl = j0 + threadIdx.x;
    tile[threadIdx.x] = jl < n ? make_float4(x[jl], y[jl], z[jl], m[jl])
                               : make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    const int cnt = (int)min((int64_t)256, n - j0);
    for (int q = ph; live && q < cnt; q += kD64Phases) {
      if (j0 + q == i) continue;
      const float4 e = tile[q];
      const double dx = (double)e.x - xi, dy = (double)e.y - yi, dz = (double)e.z - zi;
      const double d2 = dx * dx + dy * dy + dz * dz;
      const double r2 = d2 + eps2;
      const double r = sqrt(r2);
      const double w = G * (double)e.w / (r2 * r);
      sx += w * dx;
      sy += w * dy;
      sz += w * dz;
      sa += w * sqrt(d2);
      sp -= G * (double)e.w / r;
    }
    __syncthreads();
  }
  part[0][ph][t] = sx;
  part[1][ph][t] = sy;
  part[2][ph][t] = sz;
  part[3][ph][t] = sa;
  part[4][ph][t] = sp;
  __syncthreads();
  if (ph == 0 && ok) {
    double o[5];
    for (int c = 0; c < 5; ++c) {
      double v = 0.0;
      for (int q = 0; q < kD64Phases; ++q) v += part[c][q][t];
      o[c] = v;
    }
    ax[k] = o[0];
    ay[k] = o[1];
    az[k] = o[2];
    if (aabs) aabs[k] = o[3];
    if (phi) phi[k] = o[4];
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

// Second-order Runge-Kutta (Heun) step, predict: x_p = x + v dt in FP64.
// Only the FP32 image of x_p is stored (for the tree and the walk); the state
// keeps x, v for the correction.
__global__ __launch_bounds__(256) void k_rk2_predict(int64_t n, const double *__restrict__ x,
                                                     const double *__restrict__ y,
                                                     const double *__restrict__ z,
                                                     const float *__restrict__ vx,
                                                     const float *__restrict__ vy,
                                                     const float *__restrict__ vz, double dt,
                                                     float *__restrict__ x32, SortedOut so) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double px = x[i] + (double)vx[i] * dt, py = y[i] + (double)vy[i] * dt,
                 pz = z[i] + (double)vz[i] * dt;
    store_position(i, n, (float)px, (float)py, (float)pz, x32, so);
  }
}

// Correct: with v_p = v + a dt (FP32), x += (v + v_p) dt/2 (FP64, the sum in
// FP64) and v += (a + a_p) dt/2 (FP32), one rounding per operation; the FP32
// image of the new x for the tree.
__global__ __launch_bounds__(256) void k_rk2_correct(
    int64_t n, double *__restrict__ x, double *__restrict__ y, double *__restrict__ z,
    float *__restrict__ vx, float *__restrict__ vy, float *__restrict__ vz,
    const float *__restrict__ ax, const float *__restrict__ ay, const float *__restrict__ az,
    const float *__restrict__ apx, const float *__restrict__ apy,
    const float *__restrict__ apz, double dt, float dt32, float hdt32,
    float *__restrict__ x32, SortedOut so) {
  const double hdt = 0.5 * dt;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float v0x = vx[i], v0y = vy[i], v0z = vz[i];
    const float a0x = ax[i], a0y = ay[i], a0z = az[i];
    const float kx = a0x * dt32, ky = a0y * dt32, kz = a0z * dt32;
    const float vpx = v0x + kx, vpy = v0y + ky, vpz = v0z + kz;
    const double sx = (double)v0x + (double)vpx, sy = (double)v0y + (double)vpy,
                 sz = (double)v0z + (double)vpz;
    const double nx = x[i] + sx * hdt, ny = y[i] + sy * hdt, nz = z[i] + sz * hdt;
    const float bx = a0x + apx[i], by = a0y + apy[i], bz = a0z + apz[i];
    const float hx = bx * hdt32, hy = by * hdt32, hz = bz * hdt32;
    x[i] = nx;
    y[i] = ny;
    z[i] = nz;
    vx[i] = v0x + hx;
    vy[i] = v0y + hy;
    vz[i] = v0z + hz;
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

void launch_direct64(int64_t n, const float *x, const float *y, const float *z,
                     const float *m, int64_t nt, const int64_t *tgt, double G, double eps,
                     double *ax, double *ay, double *az, double *aabs, double *phi,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_direct64, dim3((unsigned)cdiv(nt, kD64Targets)), dim3(256), 0, st, n, x,
                     y, z, m, nt, tgt, G, eps * eps, ax, ay, az, aabs, phi);
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

void launch_rk2_predict(int64_t n, const double *x, const double *y, const double *z,
                        const float *vx, const float *vy, const float *vz, double dt,
                        float *x32, SortedOut so, hipStream_t st) {
  hipLaunchKernelGGL(k_rk2_predict, dim3(grid_1d(n)), dim3(256), 0, st, n, x, y, z, vx, vy, vz,
                     dt, x32, so);
}

void launch_rk2_correct(int64_t n, double *x, double *y, double *z, float *vx, float *vy,
                        float *vz, const float *ax, const float *ay, const float *az,
                        const float *apx, const float *apy, const float *apz, double dt,
                        float *x32, SortedOut so, hipStream_t st) {
  hipLaunchKernelGGL(k_rk2_correct, dim3(grid_1d(n)), dim3(256), 0, st, n, x, y, z, vx, vy, vz,
                     ax, ay, az, apx, apy, apz, dt, (float)dt, (float)(0.5 * dt), x32, so);
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
