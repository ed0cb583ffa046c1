// k_keyorder.hip -- the block-step state in key order within one nbody_step
// call.
//
// The state arrays the caller passes are in caller order, while every
// per-particle pass of a block step (drift, the queue flags, the walk's
// results, the closing kick, the group bounds) works on the tree's sorted
// order. Inside one call the state is therefore kept in key order: gathered
// once on entry, permuted at every rebuild from the old key order into the
// new one (particles move little between rebuilds, so these reads are nearly
// in order), and scattered back to caller order on exit. The arithmetic of a
// step does not depend on where a particle's values are stored, so results
// are bit-identical to a caller-order step.
#include "nbody_internal.h"

namespace nb {

namespace {
int ko_grid(int64_t n) {
  int64_t g = cdiv(n, 256 * 4);
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  return (int)g;
}
}  // namespace

__global__ __launch_bounds__(256) void k_ko_gather(
    int64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const float *__restrict__ vx, const float *__restrict__ vy,
    const float *__restrict__ vz, const float *__restrict__ ax, const float *__restrict__ ay,
    const float *__restrict__ az, const float *__restrict__ m,
    const int8_t *__restrict__ level, KoSet k, const unsigned long long *__restrict__ skip) {
  if (skip && skip[0] == skip[1]) return;  // the set holds this state already
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t o = k.pt[s];
    k.x[s] = x[o];
    k.y[s] = y[o];
    k.z[s] = z[o];
    k.vx[s] = vx[o];
    k.vy[s] = vy[o];
    k.vz[s] = vz[o];
    k.ax[s] = ax[o];
    k.ay[s] = ay[o];
    k.az[s] = az[o];
    k.m[s] = m[o];
    k.lv[s] = level[o];
  }
}

__global__ __launch_bounds__(256) void k_ko_scatter(int64_t n, KoSet k, double *__restrict__ x,
                                                    double *__restrict__ y, double *__restrict__ z,
                                                    float *__restrict__ vx, float *__restrict__ vy,
                                                    float *__restrict__ vz, float *__restrict__ ax,
                                                    float *__restrict__ ay, float *__restrict__ az,
                                                    int8_t *__restrict__ level) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t o = k.pt[s];
    x[o] = k.x[s];
    y[o] = k.y[s];
    z[o] = k.z[s];
    vx[o] = k.vx[s];
    vy[o] = k.vy[s];
    vz[o] = k.vz[s];
    ax[o] = k.ax[s];
    ay[o] = k.ay[s];
    az[o] = k.az[s];
    level[o] = k.lv[s];
  }
}

__global__ __launch_bounds__(256) void k_ko_permute(int64_t n, const uint32_t *__restrict__ perm,
                                                    KoSet f, KoSet t) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t o = perm[s];
    t.x[s] = f.x[o];
    t.y[s] = f.y[o];
    t.z[s] = f.z[o];
    t.vx[s] = f.vx[o];
    t.vy[s] = f.vy[o];
    t.vz[s] = f.vz[o];
    t.ax[s] = f.ax[o];
    t.ay[s] = f.ay[o];
    t.az[s] = f.az[o];
    t.m[s] = f.m[o];
    t.pt[s] = f.pt[o];
    t.lv[s] = f.lv[o];
  }
}

namespace {
// splitmix64's finaliser (Steele, Lea and Flood 2014).
__device__ __forceinline__ unsigned long long state_mix(unsigned long long x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

__device__ __forceinline__ unsigned long long pack2(float a, float b) {
  return (unsigned long long)__float_as_uint(a) | ((unsigned long long)__float_as_uint(b) << 32);
}
}  // namespace

// Sum over particles of a chained mix of the particle's index and the bit
// patterns of its values (order-free, so the result does not depend on the
// launch); one atomic per workgroup.
__global__ __launch_bounds__(256) void k_ko_hash(
    int64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const float *__restrict__ vx, const float *__restrict__ vy,
    const float *__restrict__ vz, const float *__restrict__ ax, const float *__restrict__ ay,
    const float *__restrict__ az, const float *__restrict__ m,
    const int8_t *__restrict__ level, unsigned long long *__restrict__ out) {
  __shared__ unsigned long long part[4];
  unsigned long long acc = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    unsigned long long h = state_mix((unsigned long long)i * 0x9e3779b97f4a7c15ull);
    h = state_mix(h ^ (unsigned long long)__double_as_longlong(x[i]));
    h = state_mix(h ^ (unsigned long long)__double_as_longlong(y[i]));
    h = state_mix(h ^ (unsigned long long)__double_as_longlong(z[i]));
    h = state_mix(h ^ pack2(vx[i], vy[i]));
    h = state_mix(h ^ pack2(vz[i], ax[i]));
    h = state_mix(h ^ pack2(ay[i], az[i]));
    h = state_mix(h ^ ((unsigned long long)__float_as_uint(m[i]) |
                   ((unsigned long long)(uint8_t)level[i] << 32)));
    acc += h;
  }
  for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if (lane_id() == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, part[0] + part[1] + part[2] + part[3]);
}

// One thread per sorted position; the first position of a run of equal keys
// sorts the run's values by caller index (insertion sort: runs are the
// particles that share one 63-bit key, usually none or a few; a run of L
// costs its thread O(L^2)).
__global__ __launch_bounds__(256) void k_ko_ties(int64_t n, const uint64_t *__restrict__ keys,
                                                 uint32_t *__restrict__ vals,
                                                 const uint32_t *__restrict__ pt_old) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j + 1 < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[j];
    if (keys[j + 1] != k || (j > 0 && keys[j - 1] == k)) continue;
    int64_t e = j + 2;
    while (e < n && keys[e] == k) ++e;
    for (int64_t a = j + 1; a < e; ++a) {
      const uint32_t v = vals[a];
      const uint32_t c = pt_old[v];
      int64_t b = a;
      while (b > j && pt_old[vals[b - 1]] > c) {
        vals[b] = vals[b - 1];
        --b;
      }
      vals[b] = v;
    }
  }
}

void launch_ko_gather(int64_t n, const double *x, const double *y, const double *z,
                      const float *vx, const float *vy, const float *vz, const float *ax,
                      const float *ay, const float *az, const float *m, const int8_t *level,
                      const KoSet &k, const unsigned long long *skip, hipStream_t st) {
  hipLaunchKernelGGL(k_ko_gather, dim3(ko_grid(n)), dim3(256), 0, st, n, x, y, z, vx, vy, vz, ax,
                     ay, az, m, level, k, skip);
}

void launch_ko_hash(int64_t n, const double *x, const double *y, const double *z,
                    const float *vx, const float *vy, const float *vz, const float *ax,
                    const float *ay, const float *az, const float *m, const int8_t *level,
                    unsigned long long *out, hipStream_t st) {
  launch_fill_u32(reinterpret_cast<uint32_t *>(out), 0u, 2, st);
  int64_t g = cdiv(n, 256 * 8);
  g = std::min<int64_t>(std::max<int64_t>(g, 1), 1024);
  hipLaunchKernelGGL(k_ko_hash, dim3((unsigned)g), dim3(256), 0, st, n, x, y, z, vx, vy, vz, ax,
                     ay, az, m, level, out);
}

void launch_ko_scatter(int64_t n, const KoSet &k, double *x, double *y, double *z, float *vx,
                       float *vy, float *vz, float *ax, float *ay, float *az, int8_t *level,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_ko_scatter, dim3(ko_grid(n)), dim3(256), 0, st, n, k, x, y, z, vx, vy,
                     vz, ax, ay, az, level);
}

void launch_ko_permute(int64_t n, const uint32_t *perm, const KoSet &from, const KoSet &to,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_ko_permute, dim3(ko_grid(n)), dim3(256), 0, st, n, perm, from, to);
}

void launch_ko_ties(int64_t n, const uint64_t *keys, uint32_t *vals, const uint32_t *pt_old,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_ko_ties, dim3(ko_grid(n)), dim3(256), 0, st, n, keys, vals, pt_old);
}

}  // namespace nb
