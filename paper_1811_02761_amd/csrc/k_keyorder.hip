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
//
// Caller order is unrelated to key order, so the entry and exit moves are
// random accesses. They go through 64-byte records (one per particle, in the
// region of the set that does not hold the state): one pass packs the
// eleven arrays into records with contiguous reads, and writes each record
// whole to its destination slot (or the next pass reads it whole from its
// source slot); the other pass moves between records and arrays in order.
// Eleven random 4- or 8-byte accesses per particle (each a partial line)
// become one access of a whole record.
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

// The hash term of caller index i and its values (a chain of mixes).
__device__ __forceinline__ unsigned long long state_hash(int64_t i, double x, double y, double z,
                                                         float vx, float vy, float vz, float ax,
                                                         float ay, float az, float m,
                                                         int8_t lv) {
  unsigned long long h = state_mix((unsigned long long)i * 0x9e3779b97f4a7c15ull);
  h = state_mix(h ^ (unsigned long long)__double_as_longlong(x));
  h = state_mix(h ^ (unsigned long long)__double_as_longlong(y));
  h = state_mix(h ^ (unsigned long long)__double_as_longlong(z));
  h = state_mix(h ^ pack2(vx, vy));
  h = state_mix(h ^ pack2(vz, ax));
  h = state_mix(h ^ pack2(ay, az));
  return state_mix(h ^ ((unsigned long long)__float_as_uint(m) |
                        ((unsigned long long)(uint8_t)lv << 32)));
}

// Sum of a 256-thread workgroup's values into part[blockIdx.x] (same-address
// atomics from thousands of workgroups would serialise; k_ko_hash_fold adds
// the partials).
__device__ __forceinline__ void block_hash_part(unsigned long long acc,
                                                unsigned long long *__restrict__ part) {
  __shared__ unsigned long long wsum[4];
  for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if (lane_id() == 0) wsum[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__device__ __forceinline__ uint32_t lo32(double v) {
  return (uint32_t)(unsigned long long)__double_as_longlong(v);
}
__device__ __forceinline__ uint32_t hi32(double v) {
  return (uint32_t)((unsigned long long)__double_as_longlong(v) >> 32);
}
__device__ __forceinline__ double dbl(uint32_t lo, uint32_t hi) {
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
}  // namespace

// Records pass through LDS in tiles of 256 (one per thread), so that each
// memory instruction moves whole 64-byte records: four consecutive lanes
// per record, instead of one lane storing or loading 16 bytes at a 64-byte
// stride. A tile row is padded to 80 bytes against LDS bank conflicts.
constexpr int kRecTile = 256;
constexpr int kRecRow = 5;  // uint4 per LDS row (4 used)

// Record of element s of a (without masses: 0), with s as its index, written
// to rec slot to[s] (to == null: slot s).
__global__ __launch_bounds__(kRecTile) void k_ko_put(int64_t n, KoSet a,
                                                     const uint32_t *__restrict__ to,
                                                     uint4 *__restrict__ rec,
                                                     const unsigned long long *__restrict__ skip) {
  if (skip && skip[0] == skip[1]) return;  // the set holds this state already
  __shared__ uint4 srec[kRecTile][kRecRow];
  __shared__ uint32_t sslot[kRecTile];
  for (int64_t t0 = blockIdx.x * (int64_t)kRecTile; t0 < n; t0 += (int64_t)gridDim.x * kRecTile) {
    const int64_t s = t0 + threadIdx.x;
    if (s < n) {
      const double x = a.x[s], y = a.y[s], z = a.z[s];
      uint4 *r = srec[threadIdx.x];
      r[0] = make_uint4(lo32(x), hi32(x), lo32(y), hi32(y));
      r[1] = make_uint4(lo32(z), hi32(z), __float_as_uint(a.vx[s]), __float_as_uint(a.vy[s]));
      r[2] = make_uint4(__float_as_uint(a.vz[s]), __float_as_uint(a.ax[s]),
                        __float_as_uint(a.ay[s]), __float_as_uint(a.az[s]));
      r[3] = make_uint4(a.m ? __float_as_uint(a.m[s]) : 0u, (uint32_t)(uint8_t)a.lv[s],
                        (uint32_t)s, 0u);
      sslot[threadIdx.x] = to ? to[s] : (uint32_t)s;
    }
    __syncthreads();
    const int cnt = (int)min((int64_t)kRecTile, n - t0);
    for (int q = threadIdx.x; q < 4 * cnt; q += kRecTile)
      rec[4 * (size_t)sslot[q >> 2] + (q & 3)] = srec[q >> 2][q & 3];
    __syncthreads();
  }
}

// Element j of b from rec slot from[j] (from == null: slot j); masses only
// where b has them; tag[j] = the record's index; with part, the workgroup's
// sum of the elements' hash terms goes to part[blockIdx.x].
__global__ __launch_bounds__(kRecTile) void k_ko_get(int64_t n, const uint4 *__restrict__ rec,
                                                     const uint32_t *__restrict__ from, KoSet b,
                                                     uint32_t *__restrict__ tag,
                                                     unsigned long long *__restrict__ part,
                                                     const unsigned long long *__restrict__ skip) {
  if (skip && skip[0] == skip[1]) return;  // the set holds this state already
  __shared__ uint4 srec[kRecTile][kRecRow];
  unsigned long long acc = 0;
  for (int64_t t0 = blockIdx.x * (int64_t)kRecTile; t0 < n; t0 += (int64_t)gridDim.x * kRecTile) {
    const int cnt = (int)min((int64_t)kRecTile, n - t0);
    for (int q = threadIdx.x; q < 4 * cnt; q += kRecTile) {
      const int64_t j = t0 + (q >> 2);
      srec[q >> 2][q & 3] = rec[4 * (size_t)(from ? from[j] : (uint32_t)j) + (q & 3)];
    }
    __syncthreads();
    const int64_t j = t0 + threadIdx.x;
    if (j < n) {
      const uint4 *r = srec[threadIdx.x];
      const uint4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
      const double x = dbl(r0.x, r0.y), y = dbl(r0.z, r0.w), z = dbl(r1.x, r1.y);
      const float vx = __uint_as_float(r1.z), vy = __uint_as_float(r1.w);
      const float vz = __uint_as_float(r2.x), ax = __uint_as_float(r2.y);
      const float ay = __uint_as_float(r2.z), az = __uint_as_float(r2.w);
      const float m = __uint_as_float(r3.x);
      const int8_t lv = (int8_t)(uint8_t)r3.y;
      b.x[j] = x;
      b.y[j] = y;
      b.z[j] = z;
      b.vx[j] = vx;
      b.vy[j] = vy;
      b.vz[j] = vz;
      b.ax[j] = ax;
      b.ay[j] = ay;
      b.az[j] = az;
      if (b.m) b.m[j] = m;
      b.lv[j] = lv;
      if (tag) tag[j] = r3.z;
      if (part) acc += state_hash(j, x, y, z, vx, vy, vz, ax, ay, az, m, lv);
    }
    __syncthreads();
  }
  if (part) block_hash_part(acc, part);
}

// *out = the sum of nb partials (one workgroup of 256).
__global__ __launch_bounds__(256) void k_ko_hash_fold(const unsigned long long *__restrict__ part,
                                                      int nb, unsigned long long *__restrict__ out) {
  __shared__ unsigned long long wsum[4];
  unsigned long long acc = 0;
  for (int b = threadIdx.x; b < nb; b += 256) acc += part[b];
  for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
  if (lane_id() == 0) wsum[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *out = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// With xyzm, also the sorted (x, y, z, m) records of the tree: the positions
// rounded to FP32, as the drift rounded them for the keys.
__global__ __launch_bounds__(256) void k_ko_permute(int64_t n, const uint32_t *__restrict__ perm,
                                                    KoSet f, KoSet t, float4 *__restrict__ xyzm) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t o = perm[s];
    const double x = f.x[o], y = f.y[o], z = f.z[o];
    const float m = f.m[o];
    if (xyzm) xyzm[s] = make_float4((float)x, (float)y, (float)z, m);
    t.x[s] = x;
    t.y[s] = y;
    t.z[s] = z;
    t.vx[s] = f.vx[o];
    t.vy[s] = f.vy[o];
    t.vz[s] = f.vz[o];
    t.ax[s] = f.ax[o];
    t.ay[s] = f.ay[o];
    t.az[s] = f.az[o];
    t.m[s] = m;
    t.pt[s] = f.pt[o];
    t.lv[s] = f.lv[o];
  }
}


// Sum over particles of a chained mix of the particle's index and the bit
// patterns of its values (order-free, so the result does not depend on the
// launch); one atomic per workgroup.
__global__ __launch_bounds__(256) void k_ko_hash(
    int64_t n, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const float *__restrict__ vx, const float *__restrict__ vy,
    const float *__restrict__ vz, const float *__restrict__ ax, const float *__restrict__ ay,
    const float *__restrict__ az, const float *__restrict__ m,
    const int8_t *__restrict__ level, unsigned long long *__restrict__ part) {
  unsigned long long acc = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    acc += state_hash(i, x[i], y[i], z[i], vx[i], vy[i], vz[i], ax[i], ay[i], az[i], m[i],
                      level[i]);
  block_hash_part(acc, part);
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

int ko_hash_parts(int64_t n) { return ko_grid(n); }

void launch_ko_gather(int64_t n, const KoSet &caller, const KoSet &k, uint4 *rec,
                      const unsigned long long *skip, hipStream_t st) {
  KoSet a = caller;
  a.pt = nullptr;
  hipLaunchKernelGGL(k_ko_put, dim3(ko_grid(n)), dim3(kRecTile), 0, st, n, a, nullptr, rec, skip);
  hipLaunchKernelGGL(k_ko_get, dim3(ko_grid(n)), dim3(kRecTile), 0, st, n, rec, k.pt, k, nullptr,
                     nullptr, skip);
}

void launch_ko_hash(int64_t n, const double *x, const double *y, const double *z,
                    const float *vx, const float *vy, const float *vz, const float *ax,
                    const float *ay, const float *az, const float *m, const int8_t *level,
                    unsigned long long *out, unsigned long long *part, hipStream_t st) {
  const int g = ko_grid(n);
  hipLaunchKernelGGL(k_ko_hash, dim3(g), dim3(256), 0, st, n, x, y, z, vx, vy, vz, ax, ay, az,
                     m, level, part);
  hipLaunchKernelGGL(k_ko_hash_fold, dim3(1), dim3(256), 0, st, part, g, out);
}

void launch_ko_scatter(int64_t n, const KoSet &k, const KoSet &caller, uint4 *rec,
                       uint32_t *inv, unsigned long long *hash, unsigned long long *part,
                       hipStream_t st) {
  KoSet b = caller;
  b.m = nullptr;  // masses do not change
  b.pt = nullptr;
  const int g = ko_grid(n);
  hipLaunchKernelGGL(k_ko_put, dim3(g), dim3(kRecTile), 0, st, n, k, k.pt, rec, nullptr);
  hipLaunchKernelGGL(k_ko_get, dim3(g), dim3(kRecTile), 0, st, n, rec, nullptr, b, inv, part,
                     nullptr);
  hipLaunchKernelGGL(k_ko_hash_fold, dim3(1), dim3(256), 0, st, part, g, hash);
}

void launch_ko_permute(int64_t n, const uint32_t *perm, const KoSet &from, const KoSet &to,
                       float4 *xyzm, hipStream_t st) {
  hipLaunchKernelGGL(k_ko_permute, dim3(ko_grid(n)), dim3(256), 0, st, n, perm, from, to,
                     xyzm);
}

void launch_ko_ties(int64_t n, const uint64_t *keys, uint32_t *vals, const uint32_t *pt_old,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_ko_ties, dim3(ko_grid(n)), dim3(256), 0, st, n, keys, vals, pt_old);
}

}  // namespace nb
