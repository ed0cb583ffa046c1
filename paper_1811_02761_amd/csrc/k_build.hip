// k_build.hip -- level-order octree and i-groups from sorted Morton keys.
//
// Tree definition (the paper's makeTree, Sec. 2.2; details it leaves open):
// a cell at level l holds the particles whose key >> 3(21-l) equals its
// prefix; it is split iff it holds more than leaf_max particles and l < 21;
// only non-empty octants become children, consecutive in octant order; cells
// are numbered by level, then by prefix.
//
// Construction without a per-level host loop. For sorted keys K and
// cpl(a, b) = number of leading octant digits K[a] and K[b] share:
//  * particle i starts a run of equal level-l prefix iff l > cpl(i-1, i);
//    let s_i = cpl(i-1, i) + 1 (s_0 = 0);
//  * the level-l cell of i holds more than W particles iff some window of
//    W+1 consecutive particles containing i shares its level-l prefix, i.e.
//    iff l <= M_i(W) = max over s in [i-W, i] of cpl(s, s+W);
//  * cells containing i exist at levels 0..D_i with D_i = min(M_i(leaf_max)
//    + 1, 21).
// So particle i starts the cells (l, i) for s_i <= l <= D_i. The level-order
// index of (l, i) is the number of cells of lower level plus the number of
// level-l cells starting before i: per-level block counts, a scan over
// blocks, and ballots inside the block give it. The window maxima use a
// sparse table (doubling) in LDS.
//
// i-groups (the particles sharing one interaction list, Sec. 1) are the cells
// holding at most group_max particles whose parent holds more (the root if
// it holds at most group_max); an oversized level-21 cell is cut into pieces
// of group_max. With group_merge, consecutive sibling group cells are joined
// greedily in octant order while the joined count stays within group_max.
// Each cell holding more than group_max particles marks the group starts
// among its children; a scan over the marked particles lists the groups in
// particle order.
#include "nbody_internal.h"

namespace nb {

constexpr int kB = kBuildThreads;
constexpr int kH = kBuildHalo;
constexpr uint32_t kGroupMark = 1u << 15;  // pinfo: particle starts a group

__device__ __forceinline__ int cpl_keys(uint64_t a, uint64_t b) {
  const uint64_t x = a ^ b;
  if (x == 0) return kMaxLevel;
  return (__clzll(x) - 1) / 3;
}

// First index j > i whose key differs from K[i] in the top 3l bits
// (galloping, then bisection). Level 0: the whole array.
__device__ uint32_t run_end(const uint64_t *__restrict__ K, uint32_t n, uint32_t i,
                            int l) {
  if (l == 0) return n;
  const int sh = 3 * (kMaxLevel - l);
  const uint64_t p = K[i] >> sh;
  uint32_t lo = i, hi = n;
  uint32_t step = 1;
  while (true) {
    const uint64_t j = (uint64_t)lo + step;
    if (j >= n) break;
    if ((K[j] >> sh) != p) {
      hi = (uint32_t)j;
      break;
    }
    lo = (uint32_t)j;
    step <<= 1;
  }
  while (hi - lo > 1) {
    const uint32_t mid = lo + (hi - lo) / 2;
    if ((K[mid] >> sh) == p)
      lo = mid;
    else
      hi = mid;
  }
  return hi;
}

// In-place doubling: t[s] <- max(t[s .. s + 2^k - 1]) for the valid prefix.
__device__ void lds_window_max(int *t, int len, int k) {
  for (int j = 0; j < k; ++j) {
    const int d = 1 << j;
    int a0 = -1, a1 = -1;
    const int t0 = threadIdx.x, t1 = threadIdx.x + kB;
    if (t0 < len) a0 = max(t[t0], t0 + d < len ? t[t0 + d] : -1);
    if (t1 < len) a1 = max(t[t1], t1 + d < len ? t[t1 + d] : -1);
    __syncthreads();
    if (t0 < len) t[t0] = a0;
    if (t1 < len) t[t1] = a1;
    __syncthreads();
  }
}

__device__ __forceinline__ int ilog2_floor(int v) { return 31 - __clz(v); }

// Pass A: per sorted particle s_i and D_i; per block and level the number of
// cells starting in the block.
__global__ __launch_bounds__(kB) void k_build_a(const uint64_t *__restrict__ K,
                                                uint32_t n, int leaf_max, int min_level,
                                                uint32_t *__restrict__ pinfo,
                                                uint32_t *__restrict__ blkcnt,
                                                uint32_t nblk) {
  __shared__ uint64_t sk[kB + 2 * kH];
  __shared__ int tL[kB + kH];
  __shared__ uint32_t wc[kLevels][kB / 64];
  const int64_t b0 = (int64_t)blockIdx.x * kB;
  for (int t = threadIdx.x; t < kB + 2 * kH; t += kB) {
    const int64_t pos = b0 - kH + t;
    sk[t] = (pos >= 0 && pos < n) ? K[pos] : 0ull;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kB + kH; t += kB) {
    const int64_t s = b0 - kH + t;
    tL[t] = (s >= 0 && s + leaf_max < n) ? cpl_keys(sk[t], sk[t + leaf_max]) : -1;
  }
  __syncthreads();
  const int kLw = ilog2_floor(leaf_max + 1);
  lds_window_max(tL, kB + kH, kLw);
  const int64_t i = b0 + threadIdx.x;
  const bool valid = i < n;
  const int li = threadIdx.x + kH;
  int s = 0, D = 0;
  if (valid) {
    s = (i == 0) ? 0 : cpl_keys(sk[li - 1], sk[li]) + 1;
    const int M = max(tL[li - leaf_max], tL[li - (1 << kLw) + 1]);
    D = max(min(M + 1, kMaxLevel), min_level);  // cells above min_level always split
    pinfo[i] = (uint32_t)s | ((uint32_t)D << 5);  // group mark (bit 15) clear
  }
  const int w = threadIdx.x >> 6;
  for (int l = 0; l < kLevels; ++l) {
    const uint64_t b = __ballot(valid && s <= l && l <= D);
    if (lane_id() == 0) wc[l][w] = (uint32_t)__popcll(b);
  }
  __syncthreads();
  if (threadIdx.x < kLevels) {
    uint32_t t = 0;
    for (int q = 0; q < kB / 64; ++q) t += wc[threadIdx.x][q];
    blkcnt[threadIdx.x * nblk + blockIdx.x] = t;
  }
}

// Exclusive scan of each row (one workgroup per row) of rows[row][0..nblk);
// the row total goes to totals[row].
__global__ __launch_bounds__(256) void k_scan_rows(uint32_t *__restrict__ rows,
                                                   uint32_t nblk,
                                                   uint32_t *__restrict__ totals) {
  __shared__ uint32_t wsum[4];
  uint32_t *row = rows + (int64_t)blockIdx.x * nblk;
  const uint32_t per = (nblk + 255) / 256;
  const uint32_t k0 = threadIdx.x * per;
  uint32_t s = 0;
  for (uint32_t k = k0; k < k0 + per && k < nblk; ++k) s += row[k];
  const uint32_t inc = wave_incl_scan(s);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 63) wsum[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
  for (int q = 0; q < 4; ++q) {
    if (q < w) off += wsum[q];
    tot += wsum[q];
  }
  uint32_t run = off + inc - s;
  for (uint32_t k = k0; k < k0 + per && k < nblk; ++k) {
    const uint32_t v = row[k];
    row[k] = run;
    run += v;
  }
  if (threadIdx.x == 0) totals[blockIdx.x] = tot;
}

// Pass C: level offsets and the cell count.
__global__ void k_build_c(const uint32_t *__restrict__ totals, DevScalars *sc,
                          int64_t cell_cap) {
  if (threadIdx.x != 0) return;
  uint32_t o = 0;
  for (int l = 0; l < kLevels; ++l) {
    sc->lvl_off[l] = o;
    o += totals[l];
  }
  sc->lvl_off[kLevels] = o;
  if ((int64_t)o > cell_cap) {
    atomicOr(&sc->status, kStCapacity);
    o = 0;
  }
  sc->ncell = o;
}

// Pass D: write every cell (l, i).
__global__ __launch_bounds__(kB) void k_build_d(
    const uint64_t *__restrict__ K, uint32_t n, const uint32_t *__restrict__ pinfo,
    const uint32_t *__restrict__ blkcnt, uint32_t nblk, const DevScalars *__restrict__ sc,
    int64_t cell_cap, int32_t *__restrict__ clevel, uint32_t *__restrict__ cpbegin,
    uint32_t *__restrict__ cpcount, int32_t *__restrict__ cfchild,
    int32_t *__restrict__ cnchild, float4 *__restrict__ nodeB,
    uint32_t *__restrict__ leafof) {
  __shared__ uint32_t wpre[kLevels][kB / 64];
  __shared__ uint32_t lvl_off[kLevels + 1];
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  const bool valid = i < n;
  const uint32_t pi = valid ? pinfo[i] : 0u;
  const int s = pi & 31, D = (pi >> 5) & 31;
  const int w = threadIdx.x >> 6;
  if (threadIdx.x <= kLevels) lvl_off[threadIdx.x] = sc->lvl_off[threadIdx.x];
  for (int l = 0; l < kLevels; ++l) {
    const uint64_t b = __ballot(valid && s <= l && l <= D);
    if (lane_id() == 0) wpre[l][w] = (uint32_t)__popcll(b);
  }
  __syncthreads();
  if (threadIdx.x < kLevels) {
    uint32_t o = 0;
    for (int q = 0; q < kB / 64; ++q) {
      const uint32_t t = wpre[threadIdx.x][q];
      wpre[threadIdx.x][q] = o;
      o += t;
    }
  }
  __syncthreads();
  const uint64_t lt = lanemask_lt();
  uint32_t idx_prev = 0;
  for (int l = 0; l < kLevels; ++l) {
    const bool bit = valid && s <= l && l <= D;
    const uint64_t b = __ballot(bit);
    if (!bit) continue;
    const uint32_t rank = blkcnt[(int64_t)l * nblk + blockIdx.x] + wpre[l][w] +
                          (uint32_t)__popcll(b & lt);
    const uint32_t idx = lvl_off[l] + rank;
    if ((int64_t)idx >= cell_cap) continue;
    if (l > s) cfchild[idx_prev] = (int32_t)idx;  // (l-1, i) is internal
    const uint32_t end = run_end(K, n, (uint32_t)i, l);
    const uint32_t cnt = end - (uint32_t)i;
    clevel[idx] = l;
    cpbegin[idx] = (uint32_t)i;
    cpcount[idx] = cnt;
    uint32_t *wB = reinterpret_cast<uint32_t *>(&nodeB[idx]);
    if (l == D) {  // leaf
      cfchild[idx] = -1;
      cnchild[idx] = 0;
      wB[2] = (uint32_t)i;
      wB[3] = cnt | kLeafBit;
      for (uint32_t p = (uint32_t)i; p < end; ++p) leafof[p] = idx;
    } else {
      int nc = 0;
      uint32_t j = (uint32_t)i;
      while (j < end) {
        j = run_end(K, n, j, l + 1);
        ++nc;
      }
      cnchild[idx] = nc;
      wB[3] = (uint32_t)nc;
      // wB[2] (first child) is written by pass E
    }
    idx_prev = idx;
  }
}

// Pass E: parents and the first-child word of internal walk nodes.
__global__ __launch_bounds__(256) void k_build_e(DevScalars *__restrict__ sc,
                                                 const int32_t *__restrict__ cfchild,
                                                 const int32_t *__restrict__ cnchild,
                                                 int32_t *__restrict__ cparent,
                                                 float4 *__restrict__ nodeB) {
  const uint32_t nc = sc->ncell;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc; c += stride) {
    if (c == 0) cparent[0] = -1;
    const int k = cnchild[c];
    if (k > 0) {
      const int32_t f = cfchild[c];
      if (f <= (int32_t)c || k > 8 || (uint32_t)(f + k) > nc) {
        atomicOr(&sc->status, kStCorrupt);
        continue;
      }
      reinterpret_cast<uint32_t *>(&nodeB[c])[2] = (uint32_t)f;
      for (int q = 0; q < k; ++q) cparent[f + q] = (int32_t)c;
    }
  }
}

__device__ __forceinline__ void mark_chunks(uint32_t *__restrict__ pinfo, uint32_t b,
                                            uint32_t cnt, uint32_t gmax) {
  for (uint32_t s = 0; s < cnt; s += gmax) pinfo[b + s] |= kGroupMark;
}

// A cell may hold a group iff it is at min_level (the system digits of a
// batch) or deeper and holds at most group_max particles or is a leaf.
__device__ __forceinline__ bool group_ok(int32_t level, uint32_t cnt, int nchild,
                                         uint32_t gmax, int min_level) {
  return level >= min_level && (cnt <= gmax || nchild == 0);
}

// Group starts: the root if it may hold a group; otherwise every cell that
// may not marks the group starts among its children (joining consecutive
// small siblings when `merge`; an over-full leaf is cut into pieces of
// group_max). Every particle is marked at most once.
__global__ __launch_bounds__(256) void k_group_mark(DevScalars *__restrict__ sc,
                                                    const int32_t *__restrict__ clevel,
                                                    const uint32_t *__restrict__ cpbegin,
                                                    const uint32_t *__restrict__ cpcount,
                                                    const int32_t *__restrict__ cfchild,
                                                    const int32_t *__restrict__ cnchild,
                                                    uint32_t gmax, int merge, int min_level,
                                                    uint32_t *__restrict__ pinfo) {
  const uint32_t nc = sc->ncell;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc;
       c += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t cnt = cpcount[c];
    const int k = cnchild[c];
    const bool ok = group_ok(clevel[c], cnt, k, gmax, min_level);
    if (c == 0 && ok) {
      mark_chunks(pinfo, cpbegin[0], cnt, gmax);
      continue;
    }
    if (ok || k == 0) continue;
    const int32_t f = cfchild[c];
    uint32_t run = 0;  // particles in the open joined group (0: none open)
    for (int q = 0; q < k; ++q) {
      const uint32_t cb = cpbegin[f + q], cc = cpcount[f + q];
      const bool cok = group_ok(clevel[f + q], cc, cnchild[f + q], gmax, min_level);
      if (cok && cc <= gmax) {
        if (merge && run > 0 && run + cc <= gmax) {
          run += cc;
        } else {
          pinfo[cb] |= kGroupMark;
          run = cc;
        }
      } else {
        run = 0;
        if (cok) mark_chunks(pinfo, cb, cc, gmax);  // an over-full (level-21) leaf
      }
    }
  }
}

// Group marks per block of kB particles.
__global__ __launch_bounds__(kB) void k_group_count(uint32_t n,
                                                    const uint32_t *__restrict__ pinfo,
                                                    uint32_t *__restrict__ gblk) {
  __shared__ uint32_t wc[kB / 64];
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  const bool mk = i < n && (pinfo[i] & kGroupMark);
  const uint64_t b = __ballot(mk);
  if (lane_id() == 0) wc[threadIdx.x >> 6] = (uint32_t)__popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int q = 0; q < kB / 64; ++q) t += wc[q];
    gblk[blockIdx.x] = t;
  }
}

// Group begins in particle order (gblk holds exclusive block offsets), and
// each particle's group (the number of group starts up to it, minus one).
__global__ __launch_bounds__(kB) void k_group_emit(uint32_t n,
                                                   const uint32_t *__restrict__ pinfo,
                                                   const uint32_t *__restrict__ gblk,
                                                   uint32_t *__restrict__ gbegin,
                                                   uint32_t *__restrict__ gid) {
  __shared__ uint32_t wc[kB / 64];
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  const bool mk = i < n && (pinfo[i] & kGroupMark);
  const uint64_t b = __ballot(mk);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) wc[w] = (uint32_t)__popcll(b);
  __syncthreads();
  uint32_t off = gblk[blockIdx.x];
  for (int q = 0; q < w; ++q) off += wc[q];
  const uint32_t before = (uint32_t)__popcll(b & lanemask_lt());
  if (mk) gbegin[off + before] = (uint32_t)i;
  if (i < n) gid[i] = off + before + (mk ? 1u : 0u) - 1u;  // particle 0 starts group 0
}

__global__ void k_group_total(const uint32_t *__restrict__ total, uint32_t n,
                              DevScalars *sc, uint32_t *__restrict__ gbegin) {
  if (threadIdx.x != 0) return;
  sc->ngroup = total[0];
  gbegin[total[0]] = n;
}

__global__ __launch_bounds__(256) void k_group_size(const DevScalars *__restrict__ sc,
                                                    const uint32_t *__restrict__ gbegin,
                                                    uint32_t *__restrict__ gcount) {
  const uint32_t ng = sc->ngroup;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < ng;
       g += (int64_t)gridDim.x * blockDim.x)
    gcount[g] = gbegin[g + 1] - gbegin[g];
}

// Batch: each group's walk starts at its system's root, the level-r cell of
// the system (one per system, numbered by system index). Sorted positions of
// system s are [off[s], off[s+1]) as in caller order.
__global__ __launch_bounds__(256) void k_group_root(const DevScalars *__restrict__ sc,
                                                    const uint32_t *__restrict__ gbegin,
                                                    const uint32_t *__restrict__ off, int nsys,
                                                    int r, uint32_t *__restrict__ groot) {
  const uint32_t ng = sc->ngroup;
  const uint32_t base = sc->lvl_off[r];
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < ng;
       g += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t b = gbegin[g];
    int lo = 0, hi = nsys;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (off[mid] <= b)
        lo = mid;
      else
        hi = mid;
    }
    groot[g] = base + (uint32_t)lo;
  }
}

void launch_build(const uint64_t *keys, int64_t n, int leaf_max, int group_max,
                  int group_merge, int nsys, int r, const Ptrs &P, const Layout &L,
                  hipStream_t st) {
  const uint32_t nblk = (uint32_t)cdiv(n, kB);
  // block rows [kLevels][nblk], then kLevels totals
  uint32_t *totals = P.blkcnt + (int64_t)kLevels * nblk;
  hipLaunchKernelGGL(k_build_a, dim3(nblk), dim3(kB), 0, st, keys, (uint32_t)n, leaf_max, r,
                     P.pinfo, P.blkcnt, nblk);
  hipLaunchKernelGGL(k_scan_rows, dim3(kLevels), dim3(256), 0, st, P.blkcnt, nblk, totals);
  hipLaunchKernelGGL(k_build_c, dim3(1), dim3(64), 0, st, totals, P.sc, L.cell_cap);
  hipLaunchKernelGGL(k_build_d, dim3(nblk), dim3(kB), 0, st, keys, (uint32_t)n, P.pinfo,
                     P.blkcnt, nblk, P.sc, L.cell_cap, P.clevel, P.cpbegin, P.cpcount,
                     P.cfchild, P.cnchild, P.nodeB, P.leafof);
  int64_t ge = cdiv(n, 256);
  if (ge > 4096) ge = 4096;
  hipLaunchKernelGGL(k_build_e, dim3(ge), dim3(256), 0, st, P.sc, P.cfchild, P.cnchild,
                     P.cparent, P.nodeB);
  // groups (the block rows are free again: reuse them for the group scan)
  uint32_t *gblk = P.blkcnt, *gtot = P.blkcnt + nblk;
  hipLaunchKernelGGL(k_group_mark, dim3(ge), dim3(256), 0, st, P.sc, P.clevel, P.cpbegin,
                     P.cpcount, P.cfchild, P.cnchild, (uint32_t)group_max, group_merge, r,
                     P.pinfo);
  hipLaunchKernelGGL(k_group_count, dim3(nblk), dim3(kB), 0, st, (uint32_t)n, P.pinfo, gblk);
  hipLaunchKernelGGL(k_scan_rows, dim3(1), dim3(256), 0, st, gblk, nblk, gtot);
  hipLaunchKernelGGL(k_group_emit, dim3(nblk), dim3(kB), 0, st, (uint32_t)n, P.pinfo, gblk,
                     P.gbegin, P.gid);
  hipLaunchKernelGGL(k_group_total, dim3(1), dim3(64), 0, st, gtot, (uint32_t)n, P.sc,
                     P.gbegin);
  hipLaunchKernelGGL(k_group_size, dim3(ge), dim3(256), 0, st, P.sc, P.gbegin, P.gcount);
  if (r > 0)
    hipLaunchKernelGGL(k_group_root, dim3(ge), dim3(256), 0, st, P.sc, P.gbegin, P.sysoff, nsys,
                       r, P.groot);
}

void launch_scan_rows(uint32_t *rows, uint32_t len, int nrows, uint32_t *totals,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_scan_rows, dim3(nrows), dim3(256), 0, st, rows, len, totals);
}

}  // namespace nb
