// k_block.hip -- individual (block) time steps with kick-drift-kick leapfrog.
//
// The paper integrates with block time steps (Sec. 1 and 4.1): particle i
// advances with dt_i = dt_max 2^-k_i, so its step boundaries are the
// multiples of 2^(10 - k_i) ticks (a tick is dt_max 2^-10). One call of the
// step loop moves the system time from tick0 to the next boundary of the
// finest occupied level:
//   opening half kick v += a dt_i/2 for the particles with a boundary at
//   tick0; drift x += v (tick - tick0) dt_tick of every particle (FP64);
//   forces for the groups holding a particle with a boundary at tick;
//   closing half kick of those particles with their old step, then a new
//   level: the smallest k (not below the alignment of the current tick) with
//   dt_k <= sqrt(2 eta eps / |a|), tested as dt_k^4 |a|^2 <= (2 eta eps)^2 in
//   FP64 (the criterion of Springel 2005, GADGET-2).
// With every particle on one level this is plain kick-drift-kick leapfrog
// operation for operation (the same FP32 kicks and FP64 drift as k_kick and
// k_drift).
#include "nbody_internal.h"

namespace nb {

constexpr int kBlkThreads = 256;
constexpr int kBlkMaxBlocks = 1024;

struct BlkTables {
  float hdt[kTickBits + 1];    // (float)(dt_k / 2)
  double lim4[kTickBits + 1];  // dt_k^4 computed as (dt_k * dt_k)^2
  double rhs;                  // (2 eta eps)^2
  double dt_tick;              // dt_max 2^-10
  int level_min, level_max;
};

BlkTables make_tables(const BlockCfg &c) {
  BlkTables t;
  for (int k = 0; k <= kTickBits; ++k) {
    const double dk = c.dt_max / (double)(1 << k);
    t.hdt[k] = (float)(0.5 * dk);
    const double d2 = dk * dk;
    t.lim4[k] = d2 * d2;
  }
  const double cc = 2.0 * c.eta * (double)c.eps;
  t.rhs = cc * cc;
  t.dt_tick = c.dt_max / (double)(1 << kTickBits);
  t.level_min = c.level_min;
  t.level_max = c.level_max;
  return t;
}

__device__ __forceinline__ int align_level(long long tick) {
  const unsigned long long t = (unsigned long long)tick & ((1ull << kTickBits) - 1);
  return t == 0 ? 0 : kTickBits - __builtin_ctzll(t);
}

// levels outside [0, 10] are reported by k_blk_scan; clamp for safe indexing
__device__ __forceinline__ int clamp_level(int k) { return min(max(k, 0), kTickBits); }

__device__ __forceinline__ bool on_boundary(long long tick, int k) {
  return (tick & ((1ll << (kTickBits - k)) - 1)) == 0;
}

__device__ int level_of(float ax, float ay, float az, const BlkTables &t, int lo) {
  const double x = ax, y = ay, z = az;
  const double xx = x * x, yy = y * y, zz = z * z;  // exact
  const double a2 = (xx + yy) + zz;
  for (int k = lo; k < t.level_max; ++k)
    if (t.lim4[k] * a2 <= t.rhs) return k;
  return t.level_max;
}

// Block-wide max and sum, written to part[2 block], part[2 block + 1];
// k_blk_fold reduces the blocks (atomics on two words from every block of a
// launch queued up behind each other: 2 x 1024 of them cost more than the
// closing kick's own traffic).
__device__ void block_fold(int kmax, uint32_t cnt, uint32_t *part) {
  __shared__ int s_max[kBlkThreads / 64];
  __shared__ uint32_t s_cnt[kBlkThreads / 64];
  for (int d = 32; d >= 1; d >>= 1) {
    kmax = max(kmax, __shfl_xor(kmax, d, 64));
    cnt += __shfl_xor(cnt, d, 64);
  }
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    s_max[w] = kmax;
    s_cnt[w] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int m = 0;
    uint32_t c = 0;
    for (int q = 0; q < kBlkThreads / 64; ++q) {
      m = max(m, s_max[q]);
      c += s_cnt[q];
    }
    part[2 * blockIdx.x] = (uint32_t)m;
    part[2 * blockIdx.x + 1] = c;
  }
}

// The blocks' maxima and counts: kmax_next = max, and (with_count) nactive
// += sum.
__global__ __launch_bounds__(256) void k_blk_fold(const uint32_t *__restrict__ part, int nb,
                                                  DevScalars *sc, int with_count) {
  uint32_t m = 0, c = 0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    m = max(m, part[2 * b]);
    c += part[2 * b + 1];
  }
  __shared__ uint32_t s_m[4], s_c[4];
  for (int d = 32; d >= 1; d >>= 1) {
    m = max(m, (uint32_t)__shfl_xor((int)m, d, 64));
    c += (uint32_t)__shfl_xor((int)c, d, 64);
  }
  if (lane_id() == 0) {
    s_m[threadIdx.x >> 6] = m;
    s_c[threadIdx.x >> 6] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < 4; ++q) {
      m = max(m, s_m[q]);
      c += s_c[q];
    }
    sc->kmax_next = max(sc->kmax_next, m);
    if (with_count) sc->nactive += c;
  }
}

__global__ void k_blk_setup(long long tick, DevScalars *sc) {
  if (threadIdx.x != 0) return;
  sc->tick = tick;
  sc->tick0 = tick;
  sc->kmax = 0;
  sc->kmax_next = 0;
  sc->nactive = 0;
  sc->nqueue = 0;
}

__global__ __launch_bounds__(kBlkThreads) void k_blk_init(int64_t n, const float *__restrict__ ax,
                                                          const float *__restrict__ ay,
                                                          const float *__restrict__ az,
                                                          int8_t *__restrict__ level,
                                                          BlkTables t, DevScalars *sc,
                                                          uint32_t *__restrict__ part) {
  const int lo = max(t.level_min, align_level(sc->tick));
  int kmax = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int k = level_of(ax[i], ay[i], az[i], t, lo);
    level[i] = (int8_t)k;
    kmax = max(kmax, k);
  }
  block_fold(kmax, 0u, part);
}

__global__ __launch_bounds__(kBlkThreads) void k_blk_scan(int64_t n,
                                                          const int8_t *__restrict__ level,
                                                          int level_min, int level_max,
                                                          DevScalars *sc, uint32_t *__restrict__ part) {
  int kmax = 0;
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int k = level[i];
    bad |= k < level_min || k > level_max;
    kmax = max(kmax, k);
  }
  if (bad) atomicOr(&sc->status, kStCorrupt);
  block_fold(min(kmax, kTickBits), 0u, part);
}

__global__ void k_blk_begin(DevScalars *sc) {
  if (threadIdx.x != 0) return;
  const long long t0 = sc->tick;
  const uint32_t k = sc->kmax_next;
  const long long s = 1ll << (kTickBits - (int)k);
  sc->tick0 = t0;
  sc->tick = (t0 / s + 1) * s;
  sc->kmax = k;
  sc->kmax_next = 0;
  sc->nactive = 0;
}

__global__ __launch_bounds__(kBlkThreads) void k_blk_open_drift(
    int64_t n, double *__restrict__ x, double *__restrict__ y, double *__restrict__ z,
    float *__restrict__ vx, float *__restrict__ vy, float *__restrict__ vz,
    const float *__restrict__ ax, const float *__restrict__ ay, const float *__restrict__ az,
    const int8_t *__restrict__ level, BlkTables t, const DevScalars *__restrict__ sc,
    float *__restrict__ x32, SortedOut so) {
  const long long t0 = sc->tick0, t1 = sc->tick;
  const double dt = (double)(t1 - t0) * t.dt_tick;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int k = clamp_level(level[i]);
    float ux = vx[i], uy = vy[i], uz = vz[i];
    if (on_boundary(t0, k)) {
      const float h = t.hdt[k];
      const float kx = ax[i] * h, ky = ay[i] * h, kz = az[i] * h;
      ux = ux + kx;
      uy = uy + ky;
      uz = uz + kz;
      vx[i] = ux;
      vy[i] = uy;
      vz[i] = uz;
    }
    const double dx = (double)ux * dt, dy = (double)uy * dt, dz = (double)uz * dt;
    const double nx = x[i] + dx, ny = y[i] + dy, nz = z[i] + dz;
    x[i] = nx;
    y[i] = ny;
    z[i] = nz;
    store_position(i, n, (float)nx, (float)ny, (float)nz, x32, so);
  }
}

// Groups holding a particle whose step ends at the current tick: one thread
// per sorted particle flags its group (same value, any order).
__global__ __launch_bounds__(kBlkThreads) void k_blk_mark(int64_t n,
                                                          const DevScalars *__restrict__ sc,
                                                          const uint32_t *__restrict__ perm,
                                                          const uint32_t *__restrict__ gid,
                                                          const int8_t *__restrict__ level,
                                                          uint32_t *__restrict__ gflag) {
  const long long tick = sc->tick;
  // four particles per trip: their index and level loads are issued together
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s0 < n; s0 += 4 * stride) {
    uint32_t p[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)  // no perm: levels in key order
      p[u] = s0 + u * stride < n ? (perm ? perm[s0 + u * stride] : (uint32_t)(s0 + u * stride))
                                 : 0u;
    int8_t lv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) lv[u] = s0 + u * stride < n ? level[p[u]] : (int8_t)0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (s0 + u * stride < n && on_boundary(tick, clamp_level(lv[u])))
        gflag[gid[s0 + u * stride]] = 1u;
  }
}

// Flagged groups per block of kQGroups groups (kQPer consecutive groups per
// thread).
constexpr int kQPer = 8;
constexpr int kQGroups = kBlkThreads * kQPer;

__device__ __forceinline__ uint32_t flagged_run(const DevScalars *__restrict__ sc, uint32_t g0,
                                                const uint32_t *__restrict__ gflag,
                                                uint32_t *bits) {
  const uint32_t ng = sc->ngroup;
  uint32_t c = 0, m = 0;
#pragma unroll
  for (int k = 0; k < kQPer; ++k) {
    const uint32_t g = g0 + (uint32_t)k;
    const bool f = g < ng && gflag[g] != 0u;
    m |= (f ? 1u : 0u) << k;
    c += f ? 1u : 0u;
  }
  *bits = m;
  return c;
}

__global__ __launch_bounds__(kBlkThreads) void k_blk_qcount(const DevScalars *__restrict__ sc,
                                                            const uint32_t *__restrict__ gflag,
                                                            uint32_t *__restrict__ blk) {
  __shared__ uint32_t wc[kBlkThreads / 64];
  const uint32_t g0 = (blockIdx.x * kBlkThreads + threadIdx.x) * kQPer;
  uint32_t bits;
  uint32_t c = flagged_run(sc, g0, gflag, &bits);
  for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
  if (lane_id() == 0) wc[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t s = 0;
    for (int q = 0; q < kBlkThreads / 64; ++q) s += wc[q];
    blk[blockIdx.x] = s;
  }
}

// The flagged groups in group order (blk holds exclusive block offsets); the
// flags are cleared for the next step.
__global__ __launch_bounds__(kBlkThreads) void k_blk_qemit(const DevScalars *__restrict__ sc,
                                                           uint32_t *__restrict__ gflag,
                                                           const uint32_t *__restrict__ blk,
                                                           uint32_t *__restrict__ order) {
  __shared__ uint32_t wc[kBlkThreads / 64];
  const uint32_t g0 = (blockIdx.x * kBlkThreads + threadIdx.x) * kQPer;
  uint32_t bits;
  const uint32_t c = flagged_run(sc, g0, gflag, &bits);
  const uint32_t inc = wave_incl_scan(c);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 63) wc[w] = inc;
  __syncthreads();
  uint32_t off = blk[blockIdx.x] + inc - c;
  for (int q = 0; q < w; ++q) off += wc[q];
  for (int k = 0; k < kQPer; ++k)
    if (bits & (1u << k)) {
      order[off++] = g0 + (uint32_t)k;
      gflag[g0 + (uint32_t)k] = 0u;
    }
}

// Exclusive scan of the per-block counts in place, by one workgroup (a
// thread per run of consecutive blocks), and the queue length.
constexpr int kQScanThreads = 1024;
__global__ __launch_bounds__(kQScanThreads) void k_blk_qscan(uint32_t *__restrict__ blk,
                                                             uint32_t nblk,
                                                             DevScalars *__restrict__ sc) {
  __shared__ uint32_t wsum[kQScanThreads / 64];
  const uint32_t per = (nblk + kQScanThreads - 1) / kQScanThreads;
  const uint32_t b0 = threadIdx.x * per, b1 = min(nblk, b0 + per);
  uint32_t s = 0;
  for (uint32_t k = b0; k < b1; ++k) s += blk[k];
  const uint32_t inc = wave_incl_scan(s);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t run = inc - s, all = 0;
  for (int q = 0; q < kQScanThreads / 64; ++q) {
    if (q < w) run += wsum[q];
    all += wsum[q];
  }
  for (uint32_t k = b0; k < b1; ++k) {
    const uint32_t v = blk[k];
    blk[k] = run;
    run += v;
  }
  if (threadIdx.x == 0) sc->nqueue = all;
}

__global__ __launch_bounds__(kBlkThreads) void k_blk_close(
    int64_t n, float *__restrict__ ax, float *__restrict__ ay, float *__restrict__ az,
    const float *__restrict__ nax, const float *__restrict__ nay,
    const float *__restrict__ naz, float *__restrict__ vx, float *__restrict__ vy,
    float *__restrict__ vz, int8_t *__restrict__ level, BlkTables t,
    float4 *__restrict__ asort, const uint32_t *__restrict__ inv, DevScalars *sc,
    uint32_t *__restrict__ part) {
  const long long t1 = sc->tick;
  const int lo = max(t.level_min, align_level(t1));
  int kmax = 0;
  uint32_t cnt = 0;
  // kCloseUnroll particles per trip, their levels loaded together (each
  // thread takes many particles; one load at a time left it waiting on memory)
  constexpr int kCloseUnroll = 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i0 < n;
       i0 += kCloseUnroll * stride) {
    int8_t lv[kCloseUnroll];
#pragma unroll
    for (int u = 0; u < kCloseUnroll; ++u) {
      const int64_t i = i0 + u * stride;
      lv[u] = i < n ? level[i] : (int8_t)0;
    }
#pragma unroll
    for (int u = 0; u < kCloseUnroll; ++u) {
      const int64_t i = i0 + u * stride;
      if (i >= n) break;
      int k = clamp_level(lv[u]);
      if (on_boundary(t1, k)) {
        const float a0 = nax[i], a1 = nay[i], a2 = naz[i];
        ax[i] = a0;
        ay[i] = a1;
        az[i] = a2;
        const float h = t.hdt[k];
        const float kx = a0 * h, ky = a1 * h, kz = a2 * h;
        vx[i] = vx[i] + kx;
        vy[i] = vy[i] + ky;
        vz[i] = vz[i] + kz;
        if (asort)  // the key-ordered mirror of caller-order state
          asort[inv[i]] = make_float4(
              a0, a1, a2, sqrt_rn(__builtin_fmaf(a2, a2, __builtin_fmaf(a1, a1, a0 * a0))));
        k = level_of(a0, a1, a2, t, lo);
        level[i] = (int8_t)k;
        ++cnt;
      }
      kmax = max(kmax, k);
    }
  }
  block_fold(kmax, cnt, part);
}

namespace {
unsigned blk_grid(int64_t n) {
  int64_t g = cdiv(n, kBlkThreads);
  if (g > kBlkMaxBlocks) g = kBlkMaxBlocks;
  if (g < 1) g = 1;
  return (unsigned)g;
}
}  // namespace

void launch_blk_setup(long long tick, DevScalars *sc, hipStream_t st) {
  hipLaunchKernelGGL(k_blk_setup, dim3(1), dim3(64), 0, st, tick, sc);
}

void launch_blk_init(int64_t n, const float *ax, const float *ay, const float *az,
                     int8_t *level, const BlockCfg &c, DevScalars *sc, uint32_t *part,
                     hipStream_t st) {
  const unsigned g = blk_grid(n);
  hipLaunchKernelGGL(k_blk_init, dim3(g), dim3(kBlkThreads), 0, st, n, ax, ay, az, level,
                     make_tables(c), sc, part);
  hipLaunchKernelGGL(k_blk_fold, dim3(1), dim3(256), 0, st, part, (int)g, sc, 0);
}

void launch_blk_scan(int64_t n, const int8_t *level, const BlockCfg &c, DevScalars *sc,
                     uint32_t *part, hipStream_t st) {
  const unsigned g = blk_grid(n);
  hipLaunchKernelGGL(k_blk_scan, dim3(g), dim3(kBlkThreads), 0, st, n, level, c.level_min,
                     c.level_max, sc, part);
  hipLaunchKernelGGL(k_blk_fold, dim3(1), dim3(256), 0, st, part, (int)g, sc, 0);
}

void launch_blk_begin(DevScalars *sc, hipStream_t st) {
  hipLaunchKernelGGL(k_blk_begin, dim3(1), dim3(64), 0, st, sc);
}

void launch_blk_open_drift(int64_t n, double *x, double *y, double *z, float *vx, float *vy,
                           float *vz, const float *ax, const float *ay, const float *az,
                           const int8_t *level, double dt_max, const DevScalars *sc,
                           float *x32, SortedOut so, hipStream_t st) {
  BlockCfg c{dt_max, 1.0, 1.0f, 0, kTickBits};
  // one particle per thread (no per-block reduction here): every thread's
  // loads are in flight at once
  int64_t g = cdiv(n, kBlkThreads);
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_blk_open_drift, dim3((unsigned)g), dim3(kBlkThreads), 0, st, n, x, y,
                     z, vx, vy, vz, ax, ay, az, level, make_tables(c), sc, x32, so);
}

void launch_blk_queue(int64_t n, const int8_t *level, const uint32_t *perm, const Ptrs &P,
                      hipStream_t st) {
  int64_t gm = cdiv(n, 4 * kBlkThreads);
  if (gm > 16384) gm = 16384;
  if (gm < 1) gm = 1;
  hipLaunchKernelGGL(k_blk_mark, dim3((unsigned)gm), dim3(kBlkThreads), 0, st, n, P.sc, perm,
                     P.gid, level, P.gflag);
  // ngroup <= n: blocks for n groups; the build's block-count buffer (free
  // outside the build) holds the per-block counts
  const uint32_t nblk = (uint32_t)cdiv(n, kQGroups);
  uint32_t *blk = P.blkcnt;
  hipLaunchKernelGGL(k_blk_qcount, dim3(nblk), dim3(kBlkThreads), 0, st, P.sc, P.gflag, blk);
  hipLaunchKernelGGL(k_blk_qscan, dim3(1), dim3(kQScanThreads), 0, st, blk, nblk, P.sc);
  hipLaunchKernelGGL(k_blk_qemit, dim3(nblk), dim3(kBlkThreads), 0, st, P.sc, P.gflag, blk,
                     P.order);
}

void launch_blk_close(int64_t n, float *ax, float *ay, float *az, const float *nax,
                      const float *nay, const float *naz, float *vx, float *vy, float *vz,
                      int8_t *level, const BlockCfg &c, float4 *asort, const uint32_t *inv,
                      DevScalars *sc, uint32_t *part, hipStream_t st) {
  // one trip of four particles per thread: a thread's loads of the levels
  // and then of the active particles' values are two round trips (a capped
  // grid left each thread eight of them)
  int64_t g = cdiv(n, 4 * kBlkThreads);
  g = std::min<int64_t>(std::max<int64_t>(g, 1), 16384);
  hipLaunchKernelGGL(k_blk_close, dim3((unsigned)g), dim3(kBlkThreads), 0, st, n, ax, ay, az,
                     nax, nay, naz, vx, vy, vz, level, make_tables(c), asort, inv, sc, part);
  hipLaunchKernelGGL(k_blk_fold, dim3(1), dim3(256), 0, st, part, (int)g, sc, 1);
}

}  // namespace nb
