// api.hip -- the C ABI (include/nbody.h): contexts, workspace, orchestration.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "nbody_internal.h"

using namespace nb;

struct nbody_ctx {
  nbody_params p;
  hipStream_t st = nullptr;
  int device = 0;
  int num_cu = 0;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  Layout L;
  Ptrs P;
  bool bound = false;
  int64_t n = 0;
  bool have_tree = false;
  uint64_t *keys = nullptr;  // sorted keys of the current tree
  uint32_t *perm = nullptr;  // sorted position -> caller index
  nbody_status sticky = NBODY_OK;
  // step statistics and rebuild controller
  int64_t steps = 0, rebuilds = 0;
  int32_t since_rebuild = 0;
  int64_t epoch = 0;      // tree builds so far (tags the spans of each tree)
  double excess_ms = 0.0;  // measured extra walk time of the current tree
  int64_t mac_walks = 0;   // walks of the current tree with the acceleration criterion
  double t_build_ms = 0.0, t_walk_ms = 0.0;  // latest measured (events)
  // timed spans: a ring of (start, end, done) events around each tree build
  // and each walk launch; a walk span's done event follows the copy of its
  // statistics to pinned host memory
  static constexpr int kSpans = 64;
  hipEvent_t ev_a[kSpans] = {}, ev_b[kSpans] = {}, ev_c[kSpans] = {};
  int span_kind[kSpans] = {};
  int64_t span_epoch[kSpans] = {};
  int sp_head = 0, sp_count = 0;
  double walk_ms_sum = 0.0, build_ms_sum = 0.0;
  int64_t walk_calls = 0, build_calls = 0;
  bool counting = false;  // accumulate the entries and interactions of every walk
  unsigned long long entries_host = 0, inter_host = 0;  // (from each walk's statistics)
  WalkStat *aux = nullptr;   // pinned, one per span (walk spans)
  bool last_queued = false;  // the last walk used the queue (block steps)
  int64_t queued_sum = 0, ngroup_sum = 0;  // groups walked / present, summed over walks
  int order = 0;       // queue order in use (params.order, or nbody_set_order)
  // P.asort mirrors (in key order, with |a|) the x component array asort_src
  // of the tree of epoch asort_epoch; set and kept within one nbody_step call
  const float *asort_src = nullptr;
  int64_t asort_epoch = -1;
  int nsys = 1, sys_r = 0;      // batch of independent systems (nbody_set_systems)
  // graph-captured steps (nbody_step_graph): one graph per step kind
  bool capturing = false;
  bool no_spans = false;  // a context on the static scratch: no events, no host copies
  hipStream_t cap_st = nullptr;  // capture and replay stream (default priority)
  hipEvent_t cap_ev[2] = {};
  hipGraphExec_t gexec[2] = {};  // [0] refit step, [1] rebuild step
  struct GraphKey {
    const void *p[10];
    int64_t n;
    double dt;
    int order, nsys;
    int64_t epoch_sys;
  } gkey[2] = {};
  int64_t sys_n = 0;            // particles of the batch
  int mlp_hidden = 0;  // hidden width of the installed cost model (0: none)
  // rebuild rule: per step kind the last walk time scaled to a fresh tree,
  // the growth I / I_ref of the last walk on the current tree, and the tick
  // and finest level of the last walk's step (block steps)
  double w0_kind[kTickBits + 1] = {};
  double growth = 1.0;
  long long last_tick = 0;
  int last_kmax = 0;
  bool block_mode = false;
  // internal cells per level of the latest tree whose counts reached the host
  // (shape of the calcNode launches): pinned copy, its event, pending flag
  uint32_t *h_istart = nullptr;
  hipEvent_t ev_istart = nullptr;
  bool istart_pending = false, have_cells = false;
  uint32_t level_cells[kMaxLevel] = {};
  // block steps inside one nbody_step call keep the state in key order in
  // set ko of the key-ordered arrays (-1: not in such a call); step_layout:
  // 0 key order for calls of kKeyedSteps steps or more, 1 always, 2 never
  int ko = -1;
  int step_layout = 0;
  // the set a key-ordered call left its state in, kept while the tree
  // (epoch) stays and the caller's arrays hash as they did on exit
  int ko_keep = -1;
  int64_t ko_keep_epoch = -1;
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Set c of the key-ordered block-step state for n particles.
KoSet ko_set(const Ptrs &P, int c, int64_t n) {
  KoSet k;
  k.x = P.kpos[c];
  k.y = k.x + n;
  k.z = k.y + n;
  k.vx = P.kvel[c];
  k.vy = k.vx + n;
  k.vz = k.vy + n;
  k.ax = P.kacc[c];
  k.ay = k.ax + n;
  k.az = k.ay + n;
  k.m = P.kmass[c];
  k.pt = P.kpt[c];
  k.lv = P.klv[c];
  return k;
}

// The region of set c as 64-byte records (4 x uint4 per particle).
uint4 *ko_records(const Ptrs &P, int c) { return reinterpret_cast<uint4 *>(P.kpos[c]); }

// Scratch for the state hash's per-workgroup partials: the block counts'
// buffer, free between launches (ko_hash_parts(n) <= ceil(n / 1024) 8-byte
// words; the buffer holds 23 ceil(n / 256) + 23 4-byte words).
unsigned long long *hash_parts(const Ptrs &P) {
  return reinterpret_cast<unsigned long long *>(P.blkcnt);
}

int device_cu_count(int *dev_out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  int cu = 0;
  if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return -1;
  if (dev_out) *dev_out = dev;
  return cu;
}

nbody_status check_params(const nbody_params *p) {
  if (!p) return NBODY_EINVAL;
  if (!(p->eps > 0.0f) || !isfinite(p->eps)) return NBODY_EINVAL;
  if (!(p->delta_acc >= 0.0f) || !isfinite(p->delta_acc)) return NBODY_EINVAL;
  if (!isfinite(p->G)) return NBODY_EINVAL;
  if (p->group_max < 1 || p->group_max > 64) return NBODY_EINVAL;
  if (p->leaf_max < 1 || p->leaf_max > p->group_max) return NBODY_EINVAL;
  if (p->compensated != 0 && p->compensated != 1) return NBODY_EINVAL;
  if (p->order < 0 || p->order > 3) return NBODY_EINVAL;
  if (p->frontier_cap != 0 &&
      (p->frontier_cap < 64 || (p->frontier_cap & (p->frontier_cap - 1)) != 0))
    return NBODY_EINVAL;
  if (p->list_tile != 0 && (p->list_tile < 64 || p->list_tile > 2048 || p->list_tile % 64))
    return NBODY_EINVAL;
  if (p->waves_per_cu < 0 || p->waves_per_cu > 32) return NBODY_EINVAL;
  if (p->checks != 0 && p->checks != 1) return NBODY_EINVAL;
  if (p->group_merge != 0 && p->group_merge != 1) return NBODY_EINVAL;
  if (p->walk_split != 0 && p->walk_split != 1 && p->walk_split != 2 && p->walk_split != 4)
    return NBODY_EINVAL;
  if (p->calcnode_sync < 0 || p->calcnode_sync > 2) return NBODY_EINVAL;
  return NBODY_OK;
}

int eff_calcnode(const nbody_params &p) {
  return p.calcnode_sync ? p.calcnode_sync : kCalcNodeLevels;
}

int eff_waves(const nbody_params &p) {
  int w = p.waves_per_cu ? p.waves_per_cu : 32;
  w = (w + kWalkWavesPerWG - 1) / kWalkWavesPerWG * kWalkWavesPerWG;
  return w;
}
// 192 entries: with the owner table, 4.5 KiB of LDS per wave lets 32 waves
// share one compute unit's 160 KiB
int eff_tile(const nbody_params &p) { return p.list_tile ? p.list_tile : 192; }
// A breadth-first walk holds at most every cell once, so the ring never needs
// more than the cell capacity (rounded up to a power of two).
int64_t eff_frontier(const nbody_params &p, int64_t cell_cap) {
  if (p.frontier_cap) return p.frontier_cap;
  int64_t f = 64;
  while (f < cell_cap && f < 16384) f <<= 1;
  return f;
}

// Kind of the block step ending at tick T (ticks of dt_max 2^-kTickBits):
// the coarsest level whose step ends there, so smaller is heavier.
int step_kind(int64_t T) {
  if (T <= 0) return 0;
  const int tz = __builtin_ctzll((unsigned long long)T);
  return kTickBits - (tz < kTickBits ? tz : kTickBits);
}

nbody_status hip_status() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? NBODY_OK : NBODY_EHIP;
}

nbody_status status_from_bits(int32_t b) {
  if (b & kStNonFinite) return NBODY_ENONFINITE;
  if (b & kStOverflow) return NBODY_EOVERFLOW;
  if (b & kStCapacity) return NBODY_ENOMEM;
  if (b & kStCorrupt) return NBODY_ECORRUPT;
  return NBODY_OK;
}

}  // namespace

namespace nb {

Layout make_layout(const nbody_params &p, int64_t n, int num_cu, bool stepping) {
  Layout L{};  // offsets not taken below stay 0 (caught by carve_complete)
  L.n_max = n;
  L.cell_cap = n + cdiv(21 * n, p.leaf_max + 1) + 2;
  L.sort_blocks = cdiv(n, kSortTile);
  L.build_blocks = cdiv(n, kBuildThreads);
  L.walk_waves = (int64_t)num_cu * eff_waves(p);
  L.num_cu = num_cu;
  L.frontier_cap = eff_frontier(p, L.cell_cap);
  // the walk's stack holds at most 512 cells per tree level (22 levels)
  L.frontier2_cap = 16384;
  L.retry_waves = 2 * kWalkWavesPerWG;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o = align256(o + bytes);
    return r;
  };
  const size_t C = (size_t)L.cell_cap, N = (size_t)n;
  L.off_scalars = take(sizeof(DevScalars));
  L.off_keysA = take(8 * N);
  L.off_keysB = take(8 * N);
  L.off_valsA = take(4 * N);
  L.off_valsB = take(4 * N);
  L.off_hist = take(4 * ((size_t)kSortRadix * L.sort_blocks + kSortRadix));
  L.off_xyzm = take(16 * N);
  L.off_x32 = take(16 * N);  // (x, y, z, m) records in caller order
  L.off_pinfo = take(4 * N);
  L.off_leafof = take(4 * N);
  L.off_blkcnt = take(4 * ((size_t)(kLevels + 1) * L.build_blocks + kLevels + 1));
  L.off_lvlblk = take(4 * ((size_t)(kLevels + 1) * L.build_blocks + kLevels + 1));
  L.off_bar = take(8 * 2 * (size_t)kBarSlots);
  L.off_clevel = take(4 * C);
  L.off_cpbegin = take(4 * C);
  L.off_cpcount = take(4 * C);
  L.off_cfchild = take(4 * C);
  L.off_cnchild = take(4 * C);
  L.off_cparent = take(4 * C);
  L.off_mom64 = take(32 * C);
  L.off_nodeA = take(16 * C);
  L.off_nodeB = take(16 * C);
  L.off_gbegin = take(4 * (N + 1));
  L.off_gcount = take(4 * N);
  L.off_gbox = take(32 * N);
  L.off_gent = take(4 * N);
  L.off_ghash = take(8 * N);
  L.off_order = take(4 * N);
  L.off_prevcnt = take(4 * N);
  L.off_frontier = take(4 * (size_t)L.walk_waves * (size_t)L.frontier_cap);
  L.off_atmp = take(12 * N);
  L.off_retry = take(4 * N);
  L.off_frontier2 = take(4 * (size_t)L.retry_waves * (size_t)L.frontier2_cap);
  L.off_feat = take(16 * N);
  L.off_target = take(4 * N);
  L.off_pred = take(4 * N);
  L.off_plast = take(4 * N);
  L.off_okeys = take(16 * N);
  L.off_qtmp = take(4 * N);
  L.off_mlpw = take(4 * (size_t)kMlpMaxParams);
  L.off_mlpm = take(4 * (size_t)kMlpMaxParams);
  L.off_mlpv = take(4 * (size_t)kMlpMaxParams);
  L.off_mlpg = take(4 * (size_t)(kMlpMaxParams + 1));
  L.off_mlppart = take(4 * (size_t)kMlpWaves * (size_t)(kMlpMaxParams + 1));
  L.off_gref = take(4 * N);
  L.off_sysoff = take(4 * (size_t)(kMaxSystems + 1));
  L.off_sysbox = take(32 * (size_t)kMaxSystems);
  L.off_groot = take(4 * N);
  L.off_inv = take(4 * N);
  L.off_asort = take(16 * N);
  // split walk: one slot per queued group while the queue is shorter than
  // 4 x the walk's wavefronts (no walk splits a longer queue)
  L.split_slots = std::max<int64_t>(1, std::min<int64_t>(4 * L.walk_waves, n));
  L.off_split = take((size_t)kSplitSlotBytes * (size_t)L.split_slots);
  L.off_gid = take(4 * N);
  L.off_gflag = take(4 * N);
  L.off_ilist = take(16 * C);
  L.off_leaves = take(8 * N);
  // the largest row scan: the build's level rows, or the internal-cell blocks
  L.off_scan = take(4 * (size_t)std::max(scan_scratch_words(L.build_blocks, kLevels + 1),
                                         scan_scratch_words(cdiv(L.cell_cap, 256), 1)));
  L.off_longcnt = take(4 * (size_t)L.build_blocks);
  L.off_longslot = take(4 * (size_t)L.build_blocks * kLevels);
  L.off_wpart = take(8 * 4 * (size_t)kStatBlocks);
  // key-ordered block-step state, two sets (none without stepping: the
  // pointers then share one empty offset and are never used); each set's
  // region, from its positions on, spans at least 64 bytes per particle: it
  // holds the 64-byte records of the entry and exit moves while the other
  // set holds the state
  const size_t K = stepping ? N : 0;
  for (int c = 0; c < 2; ++c) {
    L.off_kpos[c] = take(24 * K);
    L.off_kvel[c] = take(12 * K);
    L.off_kacc[c] = take(12 * K);
    L.off_kmass[c] = take(4 * K);
    L.off_kpt[c] = take(4 * K);
    L.off_klv[c] = take(K);
    const size_t used = o - L.off_kpos[c];
    if (used < 64 * K) take(64 * K - used);
  }
  L.total = o;
  return L;
}

// Every buffer but the scalars lies past offset 0: a pointer that is null or
// at the workspace base was never carved (a missing layout entry).
bool carve_complete(const Ptrs &P, const void *base) {
  static_assert(sizeof(Ptrs) % sizeof(void *) == 0, "Ptrs holds pointers only");
  void *slots[sizeof(Ptrs) / sizeof(void *)];
  memcpy(slots, &P, sizeof(Ptrs));
  for (size_t i = 1; i < sizeof(Ptrs) / sizeof(void *); ++i)
    if (slots[i] == nullptr || slots[i] == base) return false;
  return slots[0] == base;
}

Ptrs carve(void *base, const Layout &L) {
  char *b = static_cast<char *>(base);
  Ptrs P{};
  P.sc = reinterpret_cast<DevScalars *>(b + L.off_scalars);
  P.keysA = reinterpret_cast<uint64_t *>(b + L.off_keysA);
  P.keysB = reinterpret_cast<uint64_t *>(b + L.off_keysB);
  P.valsA = reinterpret_cast<uint32_t *>(b + L.off_valsA);
  P.valsB = reinterpret_cast<uint32_t *>(b + L.off_valsB);
  P.hist = reinterpret_cast<uint32_t *>(b + L.off_hist);
  P.xyzm = reinterpret_cast<float4 *>(b + L.off_xyzm);
  P.x32 = reinterpret_cast<float *>(b + L.off_x32);
  P.pinfo = reinterpret_cast<uint32_t *>(b + L.off_pinfo);
  P.leafof = reinterpret_cast<uint32_t *>(b + L.off_leafof);
  P.blkcnt = reinterpret_cast<uint32_t *>(b + L.off_blkcnt);
  P.lvlblk = reinterpret_cast<uint32_t *>(b + L.off_lvlblk);
  P.bar = reinterpret_cast<unsigned long long *>(b + L.off_bar);
  P.clevel = reinterpret_cast<int32_t *>(b + L.off_clevel);
  P.cpbegin = reinterpret_cast<uint32_t *>(b + L.off_cpbegin);
  P.cpcount = reinterpret_cast<uint32_t *>(b + L.off_cpcount);
  P.cfchild = reinterpret_cast<int32_t *>(b + L.off_cfchild);
  P.cnchild = reinterpret_cast<int32_t *>(b + L.off_cnchild);
  P.cparent = reinterpret_cast<int32_t *>(b + L.off_cparent);
  P.mom64 = reinterpret_cast<double4 *>(b + L.off_mom64);
  P.nodeA = reinterpret_cast<float4 *>(b + L.off_nodeA);
  P.nodeB = reinterpret_cast<float4 *>(b + L.off_nodeB);
  P.gbegin = reinterpret_cast<uint32_t *>(b + L.off_gbegin);
  P.gcount = reinterpret_cast<uint32_t *>(b + L.off_gcount);
  P.gbox = reinterpret_cast<float4 *>(b + L.off_gbox);
  P.gent = reinterpret_cast<uint32_t *>(b + L.off_gent);
  P.ghash = reinterpret_cast<unsigned long long *>(b + L.off_ghash);
  P.order = reinterpret_cast<uint32_t *>(b + L.off_order);
  P.prevcnt = reinterpret_cast<uint32_t *>(b + L.off_prevcnt);
  P.frontier = reinterpret_cast<uint32_t *>(b + L.off_frontier);
  P.atmp = reinterpret_cast<float *>(b + L.off_atmp);
  P.retry = reinterpret_cast<uint32_t *>(b + L.off_retry);
  P.frontier2 = reinterpret_cast<uint32_t *>(b + L.off_frontier2);
  P.feat = reinterpret_cast<float4 *>(b + L.off_feat);
  P.target = reinterpret_cast<float *>(b + L.off_target);
  P.pred = reinterpret_cast<float *>(b + L.off_pred);
  P.plast = reinterpret_cast<uint32_t *>(b + L.off_plast);
  P.okeys = reinterpret_cast<uint64_t *>(b + L.off_okeys);
  P.qtmp = reinterpret_cast<uint32_t *>(b + L.off_qtmp);
  P.mlpw = reinterpret_cast<float *>(b + L.off_mlpw);
  P.mlpm = reinterpret_cast<float *>(b + L.off_mlpm);
  P.mlpv = reinterpret_cast<float *>(b + L.off_mlpv);
  P.mlpg = reinterpret_cast<float *>(b + L.off_mlpg);
  P.mlppart = reinterpret_cast<float *>(b + L.off_mlppart);
  P.gref = reinterpret_cast<uint32_t *>(b + L.off_gref);
  P.sysoff = reinterpret_cast<uint32_t *>(b + L.off_sysoff);
  P.sysbox = reinterpret_cast<double4 *>(b + L.off_sysbox);
  P.groot = reinterpret_cast<uint32_t *>(b + L.off_groot);
  P.inv = reinterpret_cast<uint32_t *>(b + L.off_inv);
  P.asort = reinterpret_cast<float4 *>(b + L.off_asort);
  P.split = reinterpret_cast<float *>(b + L.off_split);
  P.gid = reinterpret_cast<uint32_t *>(b + L.off_gid);
  P.gflag = reinterpret_cast<uint32_t *>(b + L.off_gflag);
  P.ilist = reinterpret_cast<uint4 *>(b + L.off_ilist);
  P.leaves = reinterpret_cast<uint2 *>(b + L.off_leaves);
  P.scan = reinterpret_cast<uint32_t *>(b + L.off_scan);
  P.longcnt = reinterpret_cast<uint32_t *>(b + L.off_longcnt);
  P.longslot = reinterpret_cast<uint32_t *>(b + L.off_longslot);
  P.wpart = reinterpret_cast<unsigned long long *>(b + L.off_wpart);
  for (int c = 0; c < 2; ++c) {
    P.kpos[c] = reinterpret_cast<double *>(b + L.off_kpos[c]);
    P.kvel[c] = reinterpret_cast<float *>(b + L.off_kvel[c]);
    P.kacc[c] = reinterpret_cast<float *>(b + L.off_kacc[c]);
    P.kmass[c] = reinterpret_cast<float *>(b + L.off_kmass[c]);
    P.kpt[c] = reinterpret_cast<uint32_t *>(b + L.off_kpt[c]);
    P.klv[c] = reinterpret_cast<int8_t *>(b + L.off_klv[c]);
  }
  return P;
}

}  // namespace nb

// Reduction of the walk statistics: sum of entries and entries x size.
// With order != nullptr only the queued groups order[0 .. nqueue) count.
__global__ __launch_bounds__(256) void k_stats(DevScalars *sc, const uint32_t *gent,
                                               const uint32_t *gcount, const uint32_t *order) {
  const uint32_t ng = order ? sc->nqueue : sc->ngroup;
  unsigned long long e = 0, it = 0;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < ng;
       q += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t g = order ? order[q] : (uint32_t)q;
    const uint32_t v = gent[g] == 0xffffffffu ? 0u : gent[g];
    e += v;
    it += (unsigned long long)v * gcount[g];
  }
  for (int d = 32; d >= 1; d >>= 1) {
    e += __shfl_xor(e, d, 64);
    it += __shfl_xor(it, d, 64);
  }
  if (lane_id() == 0) {
    atomicAdd(&sc->entries_total, e);
    atomicAdd(&sc->inter_total, it);
  }
}

// Running totals over walks while counting is on (nbody_timing).
__global__ __launch_bounds__(256) void k_stats_accum(DevScalars *sc, const uint32_t *gent,
                                                     const uint32_t *gcount,
                                                     const uint32_t *order) {
  const uint32_t ng = order ? sc->nqueue : sc->ngroup;
  unsigned long long e = 0, it = 0;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < ng;
       q += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t g = order ? order[q] : (uint32_t)q;
    const uint32_t v = gent[g] == 0xffffffffu ? 0u : gent[g];
    e += v;
    it += (unsigned long long)v * gcount[g];
  }
  for (int d = 32; d >= 1; d >>= 1) {
    e += __shfl_xor(e, d, 64);
    it += __shfl_xor(it, d, 64);
  }
  if (lane_id() == 0) {
    atomicAdd(&sc->entries_acc, e);
    atomicAdd(&sc->inter_acc, it);
  }
}

__global__ void k_acc_zero(DevScalars *sc) {
  sc->entries_acc = 0;
  sc->inter_acc = 0;
}

__global__ void k_stats_zero(DevScalars *sc) {
  sc->entries_total = 0;
  sc->inter_total = 0;
}

__global__ void k_scalars_init(DevScalars *sc) {
  sc->status = 0;
  sc->ncell = 0;
  sc->ngroup = 0;
  sc->queue_head = 0;
  for (int l = 0; l <= kLevels; ++l) sc->lvl_off[l] = 0;
  sc->entries_total = 0;
  sc->inter_total = 0;
  sc->entries_acc = 0;
  sc->inter_acc = 0;
  sc->tick = 0;
  sc->tick0 = 0;
  sc->kmax = 0;
  sc->kmax_next = 0;
  sc->nqueue = 0;
  sc->nactive = 0;
  sc->bar_epoch = 0;
  for (int l = 0; l <= kLevels; ++l) sc->istart[l] = 0;
  sc->nleaf = 0;
}

// FP32 image of FP64 positions with the masses, (x, y, z, m) records in
// caller order, into x32.
__global__ __launch_bounds__(256) void k_to_f32(int64_t n, const double *x, const double *y,
                                                const double *z, const float *m,
                                                float4 *x32) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x32[i] = make_float4((float)x[i], (float)y[i], (float)z[i], m[i]);
}

namespace {

nbody_status pre(nbody_ctx *ctx) {
  if (!ctx) return NBODY_EINVAL;
  if (ctx->sticky != NBODY_OK) return ctx->sticky;
  if (!ctx->bound) return NBODY_ENOMEM;
  return NBODY_OK;
}

WalkCfg walk_cfg(const nbody_ctx *ctx, bool bootstrap, bool queued) {
  WalkCfg c;
  c.G = ctx->p.G;
  c.eps = ctx->p.eps;
  c.bootstrap = bootstrap ? 1 : 0;
  c.compensated = ctx->p.compensated;
  c.list_tile = eff_tile(ctx->p);
  c.frontier_cap = (int)ctx->L.frontier_cap;
  c.hash = ctx->p.checks != 0;
  c.waves_per_cu = eff_waves(ctx->p);
  c.num_cu = ctx->num_cu;
  c.use_order = queued ? 1 : 0;
  c.frontier2_cap = ctx->L.frontier2_cap;
  c.retry_waves = ctx->L.retry_waves;
  c.batch = ctx->sys_r > 0;
  c.asort_out = false;
  c.split = ctx->p.walk_split;
  c.split_slots = ctx->L.split_slots;
  return c;
}

void harvest(nbody_ctx *ctx, bool block);

// While a step is being captured into a graph there are no spans (no events,
// no copies to the host): span_begin returns -1 and the rest do nothing.
int span_begin(nbody_ctx *ctx, int kind) {
  if (ctx->capturing || ctx->no_spans) return -1;
  if (ctx->sp_count == nbody_ctx::kSpans) harvest(ctx, true);
  const int i = (ctx->sp_head + ctx->sp_count) % nbody_ctx::kSpans;
  ctx->span_kind[i] = kind;
  ctx->span_epoch[i] = ctx->epoch;
  (void)hipEventRecord(ctx->ev_a[i], ctx->st);
  return i;
}

void span_end(nbody_ctx *ctx, int i) {
  if (i < 0) return;
  (void)hipEventRecord(ctx->ev_b[i], ctx->st);
  ctx->sp_count++;
}

// After the end event of walk span i: its statistics to pinned memory, then
// the span's done event.
void span_stats(nbody_ctx *ctx, int i, bool queued, bool record) {
  if (i < 0) return;
  launch_walk_stat(queued, record, ctx->P, ctx->st);
  (void)hipMemcpyAsync(&ctx->aux[i], &ctx->P.sc->wstat, sizeof(WalkStat),
                       hipMemcpyDeviceToHost, ctx->st);
}

void span_done(nbody_ctx *ctx, int i) {
  if (i >= 0) (void)hipEventRecord(ctx->ev_c[i], ctx->st);
}

int pending_walks(const nbody_ctx *ctx) {
  int k = 0;
  for (int j = 0; j < ctx->sp_count; ++j)
    k += ctx->span_kind[(ctx->sp_head + j) % nbody_ctx::kSpans] == 1;
  return k;
}

// Fold finished spans into the timers and the rebuild controller (oldest
// first); with block, wait for the oldest pending span.
void harvest(nbody_ctx *ctx, bool block) {
  bool first = true;
  while (ctx->sp_count > 0) {
    const int i = ctx->sp_head;
    if (block && first) {
      if (hipEventSynchronize(ctx->ev_c[i]) != hipSuccess) return;
    } else if (hipEventQuery(ctx->ev_c[i]) != hipSuccess) {
      return;
    }
    first = false;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->ev_a[i], ctx->ev_b[i]) == hipSuccess) {
      if (ctx->span_kind[i] == 0) {
        ctx->t_build_ms = ms;
        ctx->build_ms_sum += ms;
        ctx->build_calls++;
      } else {
        const WalkStat &w = ctx->aux[i];
        ctx->t_walk_ms = ms;
        ctx->walk_ms_sum += ms;
        ctx->walk_calls++;
        ctx->queued_sum += w.queued;
        ctx->ngroup_sum += w.ngroup;
        if (ctx->counting) {
          ctx->entries_host += w.entries;
          ctx->inter_host += w.inter;
        }
        // extra time of this walk over a walk on the fresh tree: the groups
        // that the reference walk also took have grown from inter_ref to
        // inter_a interactions; the whole walk is taken to have grown alike
        const double g = (w.inter_ref > 0 && w.inter_ref < w.inter_a)
                             ? (double)w.inter_a / (double)w.inter_ref
                             : 1.0;
        if (ctx->span_epoch[i] == ctx->epoch) {
          ctx->excess_ms += ms * (1.0 - 1.0 / g);
          ctx->growth = g;
        }
        ctx->w0_kind[ctx->block_mode ? step_kind(w.tick) : 0] = ms / g;
        ctx->last_tick = w.tick;
        ctx->last_kmax = (int)w.kmax;
      }
    }
    ctx->sp_head = (ctx->sp_head + 1) % nbody_ctx::kSpans;
    ctx->sp_count--;
  }
}

// Internal cells per level of the latest tree whose counts have reached the
// host, or null (calcNode then launches every level).
const uint32_t *moment_plan(nbody_ctx *ctx) {
  if (ctx->istart_pending && hipEventQuery(ctx->ev_istart) == hipSuccess) {
    for (int l = 0; l < kMaxLevel; ++l)
      ctx->level_cells[l] = ctx->h_istart[l + 1] - ctx->h_istart[l];
    ctx->istart_pending = false;
    ctx->have_cells = true;
  }
  return ctx->have_cells ? ctx->level_cells : nullptr;
}

// The (x, y, z, m) records of x32 as coordinates.
Coords records(const float *x32) { return Coords{x32, x32 + 1, x32 + 2, x32 + 3, 4}; }

nbody_status do_build(nbody_ctx *ctx, int64_t n, const Coords &c) {
  const Ptrs &P = ctx->P;
  if (ctx->sys_r > 0 && n != ctx->sys_n) return NBODY_EINVAL;  // not the configured batch
  // key-ordered block steps: c holds the drifted positions in the old key
  // order, so the sort's values are old slots; the state is permuted below
  const bool ko = ctx->ko >= 0;
  // a mirror of the old tree's key order is carried over to the new one
  const bool remap = !ko && ctx->asort_src && ctx->asort_epoch == ctx->epoch &&
                     ctx->have_tree && ctx->n == n;
  ctx->epoch++;
  ctx->excess_ms = 0.0;
  ctx->growth = 1.0;
  ctx->mac_walks = 0;
  const int sp = span_begin(ctx, 0);
  if (ctx->sys_r > 0) {
    // (block counts are free before the build)
    launch_sys_keys(c, n, ctx->nsys, ctx->sys_r, P, P.blkcnt,
                    (int64_t)(kLevels + 1) * ctx->L.build_blocks + kLevels + 1, ctx->st);
  } else {
    launch_bbox(c, n, P.sc, P.blkcnt, ctx->st);  // (block counts are free before the build)
    launch_keys(c, n, P.sc, P.keysA, P.valsA, ctx->st);
  }
  uint64_t *ks;
  uint32_t *pm;
  launch_sort(n, P.keysA, P.valsA, P.keysB, P.valsB, P.hist, ctx->st, &ks, &pm);
  if (ko) launch_ko_ties(n, ks, pm, P.kpt[ctx->ko], ctx->st);  // equal keys: caller order
  // (key order: the state permute below writes the sorted records)
  if (!ko) launch_gather(c, pm, n, P.xyzm, ctx->st);
  if (remap) {  // (before inv is rewritten; okeys is free outside a walk)
    launch_asort_remap(pm, P.inv, n, P.asort, reinterpret_cast<float4 *>(P.okeys), ctx->st);
    ctx->asort_epoch = ctx->epoch;
  }
  if (ko) {
    const int c1 = 1 - ctx->ko;
    launch_ko_permute(n, pm, ko_set(P, ctx->ko, n), ko_set(P, c1, n), P.xyzm, ctx->st);
    ctx->ko = c1;
  } else {
    launch_invert(pm, n, P.inv, ctx->st);
  }
  launch_build(ks, n, ctx->p.leaf_max, ctx->p.group_max, ctx->p.group_merge, ctx->nsys,
               ctx->sys_r, P, ctx->L, ctx->st);
  const uint32_t *plan = moment_plan(ctx);
  if (ctx->h_istart && !ctx->capturing && !ctx->istart_pending) {
    // this tree's counts for the later refits (read once the copy has landed)
    (void)hipMemcpyAsync(ctx->h_istart, &P.sc->istart, sizeof(uint32_t) * (kLevels + 1),
                         hipMemcpyDeviceToHost, ctx->st);
    (void)hipEventRecord(ctx->ev_istart, ctx->st);
    ctx->istart_pending = true;
  }
  launch_moments(n, ctx->p.G, P, ctx->L, eff_calcnode(ctx->p), plan, ctx->st);
  span_end(ctx, sp);
  span_done(ctx, sp);
  launch_fill_u32(P.gref, 0u, n, ctx->st);
  // previous list lengths are those of walks on the current tree (0: none yet)
  launch_fill_u32(P.plast, 0u, n, ctx->st);
  ctx->keys = ks;
  // the tree's permutation (sorted position -> caller index)
  ctx->perm = ko ? P.kpt[ctx->ko] : pm;
  ctx->n = n;
  ctx->have_tree = true;
  return hip_status();
}

nbody_status do_refit(nbody_ctx *ctx, const Coords &c) {
  launch_gather(c, ctx->perm, ctx->n, ctx->P.xyzm, ctx->st);
  launch_moments(ctx->n, ctx->p.G, ctx->P, ctx->L, eff_calcnode(ctx->p), moment_plan(ctx),
                 ctx->st);
  return hip_status();
}

// Refit after a drift that wrote the key-ordered positions itself.
nbody_status do_refit_sorted(nbody_ctx *ctx) {
  launch_moments(ctx->n, ctx->p.G, ctx->P, ctx->L, eff_calcnode(ctx->p), moment_plan(ctx),
                 ctx->st);
  return hip_status();
}

// Within a step: mirror the state's accelerations in key order for the
// current tree (after a rebuild, or at the first step of a call).
void ensure_asort(nbody_ctx *ctx, const nbody_state *st) {
  if (ctx->asort_src == st->ax && ctx->asort_epoch == ctx->epoch) return;
  launch_asort_gather(ctx->perm, ctx->n, st->ax, st->ay, st->az, ctx->P.asort, ctx->st);
  ctx->asort_src = st->ax;
  ctx->asort_epoch = ctx->epoch;
}

// Drift output: the key-ordered array of the current tree when the step
// refits it (same particle set), else the caller-order FP32 image.
SortedOut drift_out(const nbody_ctx *ctx, const nbody_state *st, bool rebuild) {
  if (rebuild || !ctx->have_tree || ctx->n != st->n) return SortedOut{nullptr, nullptr, st->m};
  return SortedOut{ctx->P.xyzm, ctx->P.inv, st->m};
}

// queued: walk only the groups order[0 .. nqueue) (block steps). With a
// cost-ordered queue the groups are first sorted by predicted cost, and after
// the walk each member keeps its list length and each group its target.
nbody_status do_calc(nbody_ctx *ctx, const float *axo, const float *ayo, const float *azo,
                     float *ax, float *ay, float *az, bool queued = false,
                     float *phi = nullptr) {
  const bool boot = axo == nullptr;
  const Ptrs &P = ctx->P;
  // key-ordered block steps: inputs and outputs are in key order (read and
  // written directly, no mirror)
  const bool ko = ctx->ko >= 0;
  const bool mirrored = !ko && axo && axo == ctx->asort_src && ctx->asort_epoch == ctx->epoch;
  const uint32_t *out_perm = ko ? nullptr : ctx->perm;
  launch_group_bounds(axo, ayo, azo, mirrored ? P.asort : nullptr, out_perm, ctx->n,
                      ctx->p.delta_acc, queued, P, ctx->st);
  // outputs over the mirrored array keep the mirror; other writes to it end it
  const bool keep_mirror = !ko && mirrored && ax == axo;
  if (!keep_mirror && ax && ax == ctx->asort_src) ctx->asort_src = nullptr;
  // the learned order needs an installed model; until then the queue is plain
  const int mode = (ctx->order == 2 && ctx->mlp_hidden == 0) ? 0 : ctx->order;
  if (mode != 0) {
    launch_cost_features(ctx->n, queued, ctx->perm, P, ctx->st);
    launch_cost_order(ctx->n, queued, mode, ctx->mlp_hidden, P, ctx->st);
  }
  const bool use_queue = queued || mode != 0;
  WalkCfg wc = walk_cfg(ctx, boot, use_queue);
  wc.asort_out = keep_mirror;
  wc.phi = phi;
  const int sp = span_begin(ctx, 1);
  launch_walk(wc, out_perm, ctx->n, ax, ay, az, P, ctx->st);
  span_end(ctx, sp);
  launch_walk_retry(wc, out_perm, ctx->n, ax, ay, az, P, ctx->st);
  // the tree's first walk with the acceleration criterion is its reference
  const bool record = !boot && ctx->mac_walks == 0;
  if (!boot) ctx->mac_walks++;
  span_stats(ctx, sp, use_queue, record);
  span_done(ctx, sp);
  ctx->last_queued = use_queue;
  if (mode != 0) launch_cost_after(ctx->n, true, ctx->perm, P, ctx->st);
  // counted from the walk statistics on the host; a captured step has none
  if (ctx->counting && ctx->capturing)
    hipLaunchKernelGGL(k_stats_accum, dim3(256), dim3(256), 0, ctx->st, P.sc, P.gent,
                       P.gcount, use_queue ? P.order : nullptr);
  return hip_status();
}

nbody_status read_scalars(nbody_ctx *ctx, DevScalars *h) {
  if (hipMemcpyAsync(h, ctx->P.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, ctx->st) !=
      hipSuccess)
    return NBODY_EHIP;
  if (hipStreamSynchronize(ctx->st) != hipSuccess) return NBODY_EHIP;
  return NBODY_OK;
}

}  // namespace

extern "C" {

int32_t nbody_abi_version(void) { return NBODY_ABI_VERSION; }

const char *nbody_strerror(nbody_status s) {
  switch (s) {
    case NBODY_OK: return "ok";
    case NBODY_EINVAL: return "invalid argument";
    case NBODY_ENOMEM: return "workspace missing or too small";
    case NBODY_EHIP: return "HIP runtime error";
    case NBODY_EOVERFLOW: return "walk frontier buffer overflow";
    case NBODY_ENOTREE: return "no tree built";
    case NBODY_ENONFINITE: return "non-finite particle data";
    case NBODY_ECORRUPT: return "internal consistency check failed";
    default: return "unknown status";
  }
}

nbody_status nbody_params_default(nbody_params *p) {
  if (!p) return NBODY_EINVAL;
  memset(p, 0, sizeof(*p));
  p->G = 1.0f;
  p->eps = 0.0078125f;      // 2^-7
  p->delta_acc = 0.001953125f;  // 2^-9
  p->leaf_max = 16;
  p->group_max = 64;
  p->group_merge = 1;
  return NBODY_OK;
}

// Rebuild rule (the paper's auto-tuned rebuild interval, Sec. 1 and 4.1,
// minimises tree-construction plus gravity time): rebuild once the measured
// extra walk time of the current tree, including the coming step's expected
// extra, reaches the build time, at a step where a rebuild is allowed.
// Exported for host-side testing.
int32_t nbody_rebuild_decide(double t_build_ms, double excess_ms, double next_excess_ms,
                             int32_t allowed, int32_t steps_since, int32_t max_interval) {
  if (steps_since <= 0) return 0;
  if (steps_since >= max_interval) return 1;
  if (!allowed) return 0;
  return excess_ms + next_excess_ms >= t_build_ms ? 1 : 0;
}

int32_t nbody_rebuild_allowed(int64_t next_tick, int64_t step_ticks) {
  if (next_tick <= 0 || step_ticks <= 0) return 1;
  return step_kind(next_tick) <= step_kind(next_tick + step_ticks) ? 1 : 0;
}

}  // extern "C"

namespace {
// Before a step's decision: wait until every walk so far is measured (the
// previous step's included). Deciding one walk behind rebuilt a step late,
// and the walk cost grows fast with the age of the tree; the wait costs little
// because the previous step's closing kernels are still queued behind its walk.
bool rebuild_due(nbody_ctx *ctx, int32_t max_interval) {
  harvest(ctx, false);
  while (pending_walks(ctx) > 0) harvest(ctx, true);
  int kind = 0, allowed = 1;
  if (ctx->block_mode) {
    // the coming step ends one step of the finest occupied level later
    const int64_t dT = (int64_t)1 << (kTickBits - std::min(std::max(ctx->last_kmax, 0), kTickBits));
    const int64_t T = ctx->last_tick + dT;
    kind = step_kind(T);
    allowed = nbody_rebuild_allowed(T, dT);
  }
  const double w0 = ctx->w0_kind[kind] > 0.0 ? ctx->w0_kind[kind] : ctx->t_walk_ms;
  const double next = w0 * (ctx->growth - 1.0);
  return nbody_rebuild_decide(ctx->t_build_ms, ctx->excess_ms, next, allowed,
                              ctx->since_rebuild, max_interval) != 0;
}
}  // namespace

extern "C" {

nbody_status nbody_create(const nbody_params *p, void *hip_stream, nbody_ctx **out) {
  if (!out) return NBODY_EINVAL;
  *out = nullptr;
  const nbody_status s = check_params(p);
  if (s != NBODY_OK) return s;
  nbody_ctx *c = new (std::nothrow) nbody_ctx();
  if (!c) return NBODY_EINVAL;
  c->p = *p;
  c->order = p->order;
  c->st = static_cast<hipStream_t>(hip_stream);
  c->num_cu = device_cu_count(&c->device);
  if (c->num_cu <= 0) {
    delete c;
    return NBODY_EHIP;
  }
  for (int i = 0; i < nbody_ctx::kSpans; ++i)
    if (hipEventCreate(&c->ev_a[i]) != hipSuccess ||
        hipEventCreate(&c->ev_b[i]) != hipSuccess ||
        hipEventCreate(&c->ev_c[i]) != hipSuccess) {
      nbody_destroy(c);
      return NBODY_EHIP;
    }
  if (hipHostMalloc((void **)&c->aux, sizeof(WalkStat) * nbody_ctx::kSpans,
                    hipHostMallocDefault) != hipSuccess) {
    c->aux = nullptr;
    nbody_destroy(c);
    return NBODY_EHIP;
  }
  if (hipHostMalloc((void **)&c->h_istart, sizeof(uint32_t) * (kLevels + 1),
                    hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_istart, hipEventDisableTiming) != hipSuccess) {
    if (c->h_istart) (void)hipHostFree(c->h_istart);
    c->h_istart = nullptr;
    nbody_destroy(c);
    return NBODY_EHIP;
  }
  *out = c;
  return NBODY_OK;
}

void nbody_destroy(nbody_ctx *ctx) {
  if (!ctx) return;
  for (int i = 0; i < nbody_ctx::kSpans; ++i) {
    if (ctx->ev_a[i]) (void)hipEventDestroy(ctx->ev_a[i]);
    if (ctx->ev_b[i]) (void)hipEventDestroy(ctx->ev_b[i]);
    if (ctx->ev_c[i]) (void)hipEventDestroy(ctx->ev_c[i]);
  }
  if (ctx->aux || ctx->h_istart) (void)hipStreamSynchronize(ctx->st);
  if (ctx->aux) (void)hipHostFree(ctx->aux);
  if (ctx->h_istart) (void)hipHostFree(ctx->h_istart);
  if (ctx->ev_istart) (void)hipEventDestroy(ctx->ev_istart);
  if (ctx->cap_st) {
    (void)hipStreamSynchronize(ctx->cap_st);
    for (int k = 0; k < 2; ++k) {
      if (ctx->gexec[k]) (void)hipGraphExecDestroy(ctx->gexec[k]);
      if (ctx->cap_ev[k]) (void)hipEventDestroy(ctx->cap_ev[k]);
    }
    (void)hipStreamDestroy(ctx->cap_st);
  }
  delete ctx;
}

nbody_status nbody_workspace_query(const nbody_params *p, int64_t n_max, size_t *bytes) {
  const nbody_status s = check_params(p);
  if (s != NBODY_OK) return s;
  if (!bytes || n_max < 1 || n_max > (int64_t)0x7fffffff / 2) return NBODY_EINVAL;
  const int cu = device_cu_count(nullptr);
  if (cu <= 0) return NBODY_EHIP;
  *bytes = make_layout(*p, n_max, cu).total;
  return NBODY_OK;
}

nbody_status nbody_bind_workspace(nbody_ctx *ctx, void *dev_ptr, size_t bytes,
                                  int64_t n_max) {
  if (!ctx || !dev_ptr || n_max < 1 || n_max > (int64_t)0x7fffffff / 2) return NBODY_EINVAL;
  if (((uintptr_t)dev_ptr & 255u) != 0) return NBODY_EINVAL;
  const Layout L = make_layout(ctx->p, n_max, ctx->num_cu);
  if (bytes < L.total) return NBODY_ENOMEM;
  if (!carve_complete(carve(dev_ptr, L), dev_ptr)) return NBODY_ECORRUPT;
  ctx->ws = dev_ptr;
  ctx->ws_bytes = bytes;
  ctx->L = L;
  ctx->P = carve(dev_ptr, L);
  ctx->bound = true;
  ctx->have_tree = false;
  ctx->sticky = NBODY_OK;
  hipLaunchKernelGGL(k_scalars_init, dim3(1), dim3(1), 0, ctx->st, ctx->P.sc);
  launch_fill_u32(ctx->P.plast, 0u, n_max, ctx->st);
  launch_fill_u32(ctx->P.gflag, 0u, n_max, ctx->st);  // cleared again by each queue build
  // grid barrier flags start below every goal
  launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->P.bar), 0u, 4 * (int64_t)kBarSlots, ctx->st);
  return hip_status();
}

nbody_status nbody_build_tree(nbody_ctx *ctx, int64_t n, const float *x, const float *y,
                              const float *z, const float *m) {
  nbody_status s = pre(ctx);
  if (s != NBODY_OK) return s;
  if (!x || !y || !z || !m || n < 1) return NBODY_EINVAL;
  if (n > ctx->L.n_max) return NBODY_ENOMEM;
  return do_build(ctx, n, Coords{x, y, z, m, 1});
}

nbody_status nbody_refit(nbody_ctx *ctx, const float *x, const float *y, const float *z,
                         const float *m) {
  nbody_status s = pre(ctx);
  if (s != NBODY_OK) return s;
  if (!ctx->have_tree) return NBODY_ENOTREE;
  if (!x || !y || !z || !m) return NBODY_EINVAL;
  return do_refit(ctx, Coords{x, y, z, m, 1});
}

nbody_status nbody_calc_acc(nbody_ctx *ctx, const float *axo, const float *ayo,
                            const float *azo, float *ax, float *ay, float *az) {
  nbody_status s = pre(ctx);
  if (s != NBODY_OK) return s;
  if (!ctx->have_tree) return NBODY_ENOTREE;
  if (!ax || !ay || !az) return NBODY_EINVAL;
  const int nnull = (axo == nullptr) + (ayo == nullptr) + (azo == nullptr);
  if (nnull != 0 && nnull != 3) return NBODY_EINVAL;
  return do_calc(ctx, axo, ayo, azo, ax, ay, az);
}

nbody_status nbody_calc_acc_pot(nbody_ctx *ctx, const float *axo, const float *ayo,
                                const float *azo, float *ax, float *ay, float *az,
                                float *phi) {
  nbody_status s = pre(ctx);
  if (s != NBODY_OK) return s;
  if (!ctx->have_tree) return NBODY_ENOTREE;
  if (!ax || !ay || !az || !phi) return NBODY_EINVAL;
  const int nnull = (axo == nullptr) + (ayo == nullptr) + (azo == nullptr);
  if (nnull != 0 && nnull != 3) return NBODY_EINVAL;
  return do_calc(ctx, axo, ayo, azo, ax, ay, az, false, phi);
}

namespace {

// Block steps (level != NULL): see nbody.h and k_block.hip.
// Block steps. With the key-ordered layout (calls of many steps) the state
// is gathered into the tree's key order on entry, permuted at every rebuild
// and scattered back on exit: every per-particle pass of a step then reads
// and writes in order. The gather and scatter cost about as much as eight
// steps save, so shorter calls work on the caller-order arrays directly,
// through the tree's permutation. Both give the same bits.
nbody_status step_block(nbody_ctx *ctx, nbody_state *st, int32_t n_steps) {
  nbody_status s;
  const int64_t n = st->n;
  const Ptrs &P = ctx->P;
  float *x32 = P.x32;
  float *tx = P.atmp, *ty = tx + n, *tz = tx + 2 * n;
  const BlockCfg bc{st->dt, st->eta, ctx->p.eps, st->level_min, st->level_max};
  DevScalars *sc = P.sc;
  const bool keyed = ctx->step_layout == 1 || (ctx->step_layout == 0 && n_steps >= kKeyedSteps);
  const unsigned to_f32_grid = (unsigned)std::min<int64_t>(cdiv(n, 1024), 8192);
  launch_blk_setup((long long)st->tick, sc, ctx->st);
  bool force_rebuild = false;
  if (!st->have_acc) {
    hipLaunchKernelGGL(k_to_f32, dim3(to_f32_grid), dim3(256), 0, ctx->st, n, st->x, st->y,
                       st->z, st->m, reinterpret_cast<float4 *>(x32));
    if ((s = do_build(ctx, n, records(x32))) != NBODY_OK) return s;
    if ((s = do_calc(ctx, nullptr, nullptr, nullptr, st->ax, st->ay, st->az)) != NBODY_OK)
      return s;
    if ((s = do_calc(ctx, st->ax, st->ay, st->az, st->ax, st->ay, st->az)) != NBODY_OK)
      return s;
    launch_blk_init(n, st->ax, st->ay, st->az, st->level, bc, sc, P.blkcnt, ctx->st);
    st->have_acc = 1;
    ctx->since_rebuild = 0;
  } else {
    launch_blk_scan(n, st->level, bc, sc, P.blkcnt, ctx->st);
    if (!ctx->have_tree || ctx->n != n) {
      // no tree of these particles: the first step builds one from the
      // drifted positions (the key-ordered layout needs one for its order
      // before that)
      force_rebuild = true;
      if (keyed) {
        hipLaunchKernelGGL(k_to_f32, dim3(to_f32_grid), dim3(256), 0, ctx->st, n, st->x, st->y,
                           st->z, st->m, reinterpret_cast<float4 *>(x32));
        if ((s = do_build(ctx, n, records(x32))) != NBODY_OK) return s;
      }
    }
  }
  if (keyed) {
    // the set the last key-ordered call left is still this state's if the
    // tree is the same and the caller's arrays hash as they did on its exit
    const bool kept = ctx->ko_keep >= 0 && ctx->ko_keep_epoch == ctx->epoch && ctx->n == n &&
                      ctx->perm == P.kpt[ctx->ko_keep];
    const int c = kept ? ctx->ko_keep : 0;
    const KoSet k0 = ko_set(P, c, n);
    if (ctx->perm != k0.pt &&
        hipMemcpyAsync(k0.pt, ctx->perm, 4 * (size_t)n, hipMemcpyDeviceToDevice, ctx->st) !=
            hipSuccess)
      return NBODY_EHIP;
    if (kept)
      launch_ko_hash(n, st->x, st->y, st->z, st->vx, st->vy, st->vz, st->ax, st->ay, st->az,
                     st->m, st->level, &sc->ko_hash[1], hash_parts(P), ctx->st);
    const KoSet caller{st->x,  st->y,  st->z,  st->vx, st->vy,   st->vz,
                       st->ax, st->ay, st->az, st->m,  nullptr, st->level};
    launch_ko_gather(n, caller, k0, ko_records(P, 1 - c), kept ? sc->ko_hash : nullptr,
                     ctx->st);
    ctx->ko = c;
    ctx->perm = k0.pt;
  }
  ctx->ko_keep = -1;
  // the state arrays of the current layout
  KoSet S{st->x, st->y, st->z, st->vx, st->vy, st->vz, st->ax, st->ay, st->az, st->m,
          nullptr, st->level};
  s = NBODY_OK;
  for (int32_t k = 0; k < n_steps && s == NBODY_OK; ++k) {
    const bool rebuild = force_rebuild ||
                         (st->rebuild_interval > 0 ? ctx->since_rebuild >= st->rebuild_interval
                                                   : rebuild_due(ctx, 64));
    force_rebuild = false;
    if (keyed) S = ko_set(P, ctx->ko, n);
    launch_blk_begin(sc, ctx->st);
    // key order: a rebuild reads the drifted positions as (x, y, z, m)
    // records in the old key order, a refit as the tree's sorted positions
    const SortedOut so = !keyed ? drift_out(ctx, st, rebuild)
                         : rebuild ? SortedOut{nullptr, nullptr, S.m}
                                   : SortedOut{P.xyzm, nullptr, S.m};
    launch_blk_open_drift(n, S.x, S.y, S.z, S.vx, S.vy, S.vz, S.ax, S.ay, S.az, S.lv, st->dt,
                          sc, x32, so, ctx->st);
    if (rebuild) {
      if ((s = do_build(ctx, n, records(x32))) != NBODY_OK) break;
      if (keyed) S = ko_set(P, ctx->ko, n);  // the state now lies in the other set
      ctx->rebuilds++;
      ctx->since_rebuild = 0;
    } else {
      if ((s = do_refit_sorted(ctx)) != NBODY_OK) break;
    }
    launch_blk_queue(n, S.lv, keyed ? nullptr : ctx->perm, P, ctx->st);
    if (!keyed) ensure_asort(ctx, st);
    if ((s = do_calc(ctx, S.ax, S.ay, S.az, tx, ty, tz, true)) != NBODY_OK) break;
    launch_blk_close(n, S.ax, S.ay, S.az, tx, ty, tz, S.vx, S.vy, S.vz, S.lv, bc,
                     keyed ? nullptr : P.asort, P.inv, sc, P.blkcnt, ctx->st);
    ctx->since_rebuild++;
    ctx->steps++;
    s = hip_status();
  }
  if (keyed) {
    // back to caller order; the tree keeps its permutation and gets its inverse
    // (and the hash a later call checks the caller's arrays against)
    const KoSet caller{st->x,  st->y,  st->z,  st->vx, st->vy,   st->vz,
                       st->ax, st->ay, st->az, st->m,  nullptr, st->level};
    launch_ko_scatter(n, ko_set(P, ctx->ko, n), caller, ko_records(P, 1 - ctx->ko), P.inv,
                      &sc->ko_hash[0], hash_parts(P), ctx->st);
    if (s == NBODY_OK) {
      ctx->ko_keep = ctx->ko;
      ctx->ko_keep_epoch = ctx->epoch;
    }
    ctx->ko = -1;
  }
  if (s != NBODY_OK) return s;
  long long tick = 0;
  if (hipMemcpyAsync(&tick, &sc->tick, sizeof(tick), hipMemcpyDeviceToHost, ctx->st) !=
          hipSuccess ||
      hipStreamSynchronize(ctx->st) != hipSuccess)
    return NBODY_EHIP;
  st->t += (double)(tick - st->tick) * (st->dt / (double)(1 << kTickBits));
  st->tick = tick;
  return NBODY_OK;
}

// Global steps of the second-order Runge-Kutta method (Heun, predict /
// correct): the tree is rebuilt (or refitted) at the predicted positions and
// refitted at the corrected ones; a_p of the predicted positions lives in
// atmp between the two walks.
nbody_status step_rk2(nbody_ctx *ctx, nbody_state *st, int32_t n_steps) {
  nbody_status s;
  const int64_t n = st->n;
  float *x32 = ctx->P.x32;
  float *px = ctx->P.atmp, *py = px + n, *pz = px + 2 * n;
  for (int32_t k = 0; k < n_steps; ++k) {
    bool rebuild = st->rebuild_interval > 0 ? ctx->since_rebuild >= st->rebuild_interval
                                            : rebuild_due(ctx, 64);
    if (ctx->n != n) rebuild = true;
    launch_rk2_predict(n, st->x, st->y, st->z, st->vx, st->vy, st->vz, st->dt, x32,
                       drift_out(ctx, st, rebuild), ctx->st);
    if (rebuild) {
      if ((s = do_build(ctx, n, records(x32))) != NBODY_OK) return s;
      ctx->rebuilds++;
      ctx->since_rebuild = 0;
    } else {
      if ((s = do_refit_sorted(ctx)) != NBODY_OK) return s;
    }
    ensure_asort(ctx, st);
    if ((s = do_calc(ctx, st->ax, st->ay, st->az, px, py, pz)) != NBODY_OK) return s;
    launch_rk2_correct(n, st->x, st->y, st->z, st->vx, st->vy, st->vz, st->ax, st->ay, st->az,
                       px, py, pz, st->dt, x32, drift_out(ctx, st, false), ctx->st);
    if ((s = do_refit_sorted(ctx)) != NBODY_OK) return s;
    // a_old of this walk is a_p: the mirror of the state's a is stale after it
    if ((s = do_calc(ctx, px, py, pz, st->ax, st->ay, st->az)) != NBODY_OK) return s;
    ctx->since_rebuild++;
    ctx->steps++;
    st->t += st->dt;
    if ((s = hip_status()) != NBODY_OK) return s;
  }
  return NBODY_OK;
}

// Global kick-drift-kick steps (no individual levels).
nbody_status step_global(nbody_ctx *ctx, nbody_state *st, int32_t n_steps) {
  nbody_status s;
  const int64_t n = st->n;
  float *x32 = ctx->P.x32;
  if (!st->have_acc) {
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)std::min<int64_t>(cdiv(n, 1024), 8192)),
                       dim3(256), 0, ctx->st, n, st->x, st->y, st->z, st->m,
                       reinterpret_cast<float4 *>(x32));
    if ((s = do_build(ctx, n, records(x32))) != NBODY_OK) return s;
    if ((s = do_calc(ctx, nullptr, nullptr, nullptr, st->ax, st->ay, st->az)) != NBODY_OK)
      return s;
    if ((s = do_calc(ctx, st->ax, st->ay, st->az, st->ax, st->ay, st->az)) != NBODY_OK)
      return s;
    st->have_acc = 1;
    ctx->since_rebuild = 0;
  }
  const float hdt = (float)(0.5 * st->dt);
  if (st->integrator == kIntRK2) return step_rk2(ctx, st, n_steps);
  for (int32_t k = 0; k < n_steps; ++k) {
    bool rebuild = st->rebuild_interval > 0 ? ctx->since_rebuild >= st->rebuild_interval
                                            : rebuild_due(ctx, 64);
    if (ctx->n != n) rebuild = true;
    launch_kick(n, st->vx, st->vy, st->vz, st->ax, st->ay, st->az, hdt, ctx->st);
    launch_drift(n, st->x, st->y, st->z, st->vx, st->vy, st->vz, st->dt, x32,
                 drift_out(ctx, st, rebuild), ctx->st);
    if (rebuild) {
      if ((s = do_build(ctx, n, records(x32))) != NBODY_OK) return s;
      ctx->rebuilds++;
      ctx->since_rebuild = 0;
    } else {
      if ((s = do_refit_sorted(ctx)) != NBODY_OK) return s;
    }
    ensure_asort(ctx, st);
    if ((s = do_calc(ctx, st->ax, st->ay, st->az, st->ax, st->ay, st->az)) != NBODY_OK)
      return s;
    launch_kick(n, st->vx, st->vy, st->vz, st->ax, st->ay, st->az, hdt, ctx->st);
    ctx->since_rebuild++;
    ctx->steps++;
    st->t += st->dt;
    if ((s = hip_status()) != NBODY_OK) return s;
  }
  return NBODY_OK;
}

}  // namespace

nbody_status nbody_step(nbody_ctx *ctx, nbody_state *st, int32_t n_steps) {
  nbody_status s = pre(ctx);
  if (s != NBODY_OK) return s;
  if (!st || n_steps < 0 || st->n < 1 || !st->x || !st->y || !st->z || !st->vx || !st->vy ||
      !st->vz || !st->m || !st->ax || !st->ay || !st->az || !(st->dt > 0.0) ||
      !isfinite(st->dt) || st->rebuild_interval < 0)
    return NBODY_EINVAL;
  if (st->level &&
      (!(st->eta > 0.0) || !isfinite(st->eta) || st->level_min < 0 ||
       st->level_min > st->level_max || st->level_max > kTickBits || st->tick < 0))
    return NBODY_EINVAL;
  if (st->integrator != kIntKDK && st->integrator != kIntRK2) return NBODY_EINVAL;
  if (st->integrator == kIntRK2 && st->level) return NBODY_EINVAL;  // global steps only
  if (st->n > ctx->L.n_max) return NBODY_ENOMEM;
  ctx->asort_src = nullptr;  // the caller may have changed the state since the last call
  ctx->block_mode = st->level != nullptr;
  s = st->level ? step_block(ctx, st, n_steps) : step_global(ctx, st, n_steps);
  ctx->asort_src = nullptr;  // and may change it before the next call
  return s;
}

nbody_status nbody_direct(nbody_ctx *ctx, int64_t n, const float *x, const float *y,
                          const float *z, const float *m, float *ax, float *ay, float *az) {
  if (!ctx) return NBODY_EINVAL;
  if (ctx->sticky != NBODY_OK) return ctx->sticky;
  if (n < 1 || !x || !y || !z || !m || !ax || !ay || !az) return NBODY_EINVAL;
  launch_direct(n, x, y, z, m, ctx->p.G, ctx->p.eps, ax, ay, az, ctx->st);
  return hip_status();
}

nbody_status nbody_direct64(nbody_ctx *ctx, int64_t n, const float *x, const float *y,
                            const float *z, const float *m, int64_t n_target,
                            const int64_t *targets, double *ax, double *ay, double *az,
                            double *aabs, double *phi) {
  if (!ctx) return NBODY_EINVAL;
  if (ctx->sticky != NBODY_OK) return ctx->sticky;
  if (n < 1 || n_target < 0 || !x || !y || !z || !m || !targets || !ax || !ay || !az)
    return NBODY_EINVAL;
  if (n_target == 0) return NBODY_OK;
  launch_direct64(n, x, y, z, m, n_target, targets, (double)ctx->p.G, (double)ctx->p.eps, ax,
                  ay, az, aabs, phi, ctx->st);
  return hip_status();
}

nbody_status nbody_sync(nbody_ctx *ctx) {
  if (!ctx) return NBODY_EINVAL;
  if (hipStreamSynchronize(ctx->st) != hipSuccess) return ctx->sticky = NBODY_EHIP;
  if (ctx->sticky != NBODY_OK || !ctx->bound) return ctx->sticky;
  int32_t bits = 0;
  if (hipMemcpy(&bits, &ctx->P.sc->status, sizeof(bits), hipMemcpyDeviceToHost) != hipSuccess)
    return ctx->sticky = NBODY_EHIP;
  ctx->sticky = status_from_bits(bits);
  harvest(ctx, false);
  return ctx->sticky;
}

nbody_status nbody_timing(nbody_ctx *ctx, int32_t enable) {
  if (!ctx) return NBODY_EINVAL;
  if (ctx->sticky != NBODY_OK) return ctx->sticky;
  if (!ctx->bound) return NBODY_ENOMEM;
  if (hipStreamSynchronize(ctx->st) != hipSuccess) return ctx->sticky = NBODY_EHIP;
  harvest(ctx, false);
  ctx->walk_ms_sum = ctx->build_ms_sum = 0.0;
  ctx->walk_calls = ctx->build_calls = 0;
  ctx->queued_sum = ctx->ngroup_sum = 0;
  ctx->counting = enable != 0;
  ctx->entries_host = ctx->inter_host = 0;
  hipLaunchKernelGGL(k_acc_zero, dim3(1), dim3(1), 0, ctx->st, ctx->P.sc);
  return hip_status();
}

nbody_status nbody_get_stats(nbody_ctx *ctx, nbody_stats *out) {
  if (!ctx || !out) return NBODY_EINVAL;
  nbody_status s = nbody_sync(ctx);
  if (s != NBODY_OK) return s;
  memset(out, 0, sizeof(*out));
  out->n = ctx->n;
  out->steps = ctx->steps;
  out->rebuilds = ctx->rebuilds;
  out->t_build_ms = ctx->t_build_ms;
  out->t_walk_ms = ctx->t_walk_ms;
  out->walk_ms_sum = ctx->walk_ms_sum;
  out->walk_calls = ctx->walk_calls;
  out->build_ms_sum = ctx->build_ms_sum;
  out->build_calls = ctx->build_calls;
  if (!ctx->have_tree) return NBODY_OK;
  hipLaunchKernelGGL(k_stats_zero, dim3(1), dim3(1), 0, ctx->st, ctx->P.sc);
  hipLaunchKernelGGL(k_stats, dim3(256), dim3(256), 0, ctx->st, ctx->P.sc, ctx->P.gent,
                     ctx->P.gcount, ctx->last_queued ? ctx->P.order : nullptr);
  DevScalars h;
  if ((s = read_scalars(ctx, &h)) != NBODY_OK) return s;
  out->ncell = h.ncell;
  out->ngroup = h.ngroup;
  out->list_entries = (int64_t)h.entries_total;
  out->interactions = (int64_t)h.inter_total;
  out->entries_sum = (int64_t)(h.entries_acc + ctx->entries_host);
  out->interactions_sum = (int64_t)(h.inter_acc + ctx->inter_host);
  out->queued = ctx->last_queued ? (int64_t)h.nqueue : (int64_t)h.ngroup;
  out->active = (int64_t)h.nactive;
  out->queued_sum = ctx->queued_sum;
  out->retried = (int64_t)h.nretry;
  out->ngroup_sum = ctx->ngroup_sum;
  return NBODY_OK;
}

nbody_status nbody_export(nbody_ctx *ctx, int32_t what, void *dst, int64_t capacity) {
  nbody_status s = pre(ctx);
  if (s != NBODY_OK) return s;
  if (!dst || capacity < 0) return NBODY_EINVAL;
  if (!ctx->have_tree) return NBODY_ENOTREE;
  DevScalars h;
  if ((s = read_scalars(ctx, &h)) != NBODY_OK) return s;
  const Ptrs &P = ctx->P;
  const int64_t n = ctx->n, nc = h.ncell, ng = h.ngroup;
  const void *src = nullptr;
  int64_t count = 0;
  size_t esz = 4;
  switch (what) {
    case NBODY_X_KEYS: src = ctx->keys; count = n; esz = 8; break;
    case NBODY_X_PERM: src = ctx->perm; count = n; break;
    case NBODY_X_LEVEL: src = P.clevel; count = nc; break;
    case NBODY_X_PBEGIN: src = P.cpbegin; count = nc; break;
    case NBODY_X_PCOUNT: src = P.cpcount; count = nc; break;
    case NBODY_X_FCHILD: src = P.cfchild; count = nc; break;
    case NBODY_X_NCHILD: src = P.cnchild; count = nc; break;
    case NBODY_X_PARENT: src = P.cparent; count = nc; break;
    case NBODY_X_NODE: src = P.nodeA; count = 4 * nc; break;
    case NBODY_X_MQ: src = nullptr; count = 2 * nc; break;
    case NBODY_X_MOM64: src = P.mom64; count = 4 * nc; esz = 8; break;
    case NBODY_X_GBEGIN: src = P.gbegin; count = ng; break;
    case NBODY_X_GCOUNT: src = P.gcount; count = ng; break;
    case NBODY_X_GBOX: src = P.gbox; count = 8 * ng; break;
    case NBODY_X_GENTRIES: src = P.gent; count = ng; break;
    case NBODY_X_GHASH: src = P.ghash; count = ng; esz = 8; break;
    case NBODY_X_XYZM: src = P.xyzm; count = 4 * n; break;
    case NBODY_X_BOX: src = P.sc->box; count = 4; esz = 8; break;
    case NBODY_X_QUEUE:
      src = P.order;
      count = ctx->last_queued ? (int64_t)h.nqueue : 0;
      break;
    case NBODY_X_FEAT: src = P.feat; count = 4 * ng; break;
    case NBODY_X_TARGET: src = P.target; count = ng; break;
    case NBODY_X_PRED: src = P.pred; count = ng; break;
    case NBODY_X_SYSBOX: src = P.sysbox; count = 4 * (int64_t)ctx->nsys; esz = 8; break;
    case NBODY_X_GROOT:
      src = P.groot;
      count = ctx->sys_r > 0 ? ng : 0;
      break;
    case NBODY_X_APRED: src = P.atmp; count = 3 * n; break;
    default: return NBODY_EINVAL;
  }
  if (capacity < count) return NBODY_ENOMEM;
  if (what == NBODY_X_MQ) {
    // nodeB holds m32, q, w0, w1: copy the first two floats of each cell
    if (hipMemcpy2DAsync(dst, 8, P.nodeB, 16, 8, (size_t)nc, hipMemcpyDeviceToDevice,
                         ctx->st) != hipSuccess)
      return NBODY_EHIP;
    return NBODY_OK;
  }
  if (count > 0 && hipMemcpyAsync(dst, src, (size_t)count * esz, hipMemcpyDeviceToDevice,
                                  ctx->st) != hipSuccess)
    return NBODY_EHIP;
  return NBODY_OK;
}


int64_t nbody_mlp_nparams(int32_t hidden) {
  return mlp_hidden_ok(hidden) ? mlp_nparams(hidden) : -1;
}

nbody_status nbody_mlp_forward(nbody_ctx *ctx, int32_t hidden, const float *w, int64_t rows,
                               const float *feat, float *y) {
  nbody_status s = pre(ctx);
  if (s != NBODY_OK) return s;
  if (!mlp_hidden_ok(hidden) || !w || !feat || !y || rows < 0 ||
      ((uintptr_t)feat & 15u) != 0)
    return NBODY_EINVAL;
  if (rows == 0) return NBODY_OK;
  launch_mlp_forward(hidden, w, rows, nullptr, reinterpret_cast<const float4 *>(feat), y,
                     ctx->st);
  return hip_status();
}

nbody_status nbody_mlp_grad(nbody_ctx *ctx, int32_t hidden, const float *w, int64_t rows,
                            const float *feat, const float *target, float *grad_loss) {
  nbody_status s = pre(ctx);
  if (s != NBODY_OK) return s;
  if (!mlp_hidden_ok(hidden) || !w || !feat || !target || !grad_loss || rows < 1 ||
      ((uintptr_t)feat & 15u) != 0)
    return NBODY_EINVAL;
  launch_mlp_grad(hidden, w, rows, reinterpret_cast<const float4 *>(feat), target,
                  ctx->P.mlppart, grad_loss, ctx->st);
  return hip_status();
}

nbody_status nbody_mlp_adam(nbody_ctx *ctx, int64_t n_params, float *w, const float *grad,
                            float *m, float *v, int32_t step, float lr, float beta1,
                            float beta2, float eps) {
  nbody_status s = pre(ctx);
  if (s != NBODY_OK) return s;
  if (!w || !grad || !m || !v || n_params < 1 || step < 1 || !(lr > 0.0f) ||
      !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return NBODY_EINVAL;
  launch_adam(n_params, w, grad, m, v, step, lr, beta1, beta2, eps, ctx->st);
  return hip_status();
}

nbody_status nbody_costmodel_train(nbody_ctx *ctx, int32_t hidden, float *w, int64_t rows,
                                   const float *feat, const float *target, int32_t steps,
                                   float lr, float *loss_out) {
  nbody_status s = pre(ctx);
  if (s != NBODY_OK) return s;
  if (!mlp_hidden_ok(hidden) || !w || !feat || !target || rows < 1 || steps < 1 ||
      !(lr > 0.0f) || ((uintptr_t)feat & 15u) != 0)
    return NBODY_EINVAL;
  const Ptrs &P = ctx->P;
  const int64_t np = mlp_nparams(hidden);
  launch_mlp_standardize(reinterpret_cast<const float4 *>(feat), rows, w, ctx->st);
  launch_fill_u32(reinterpret_cast<uint32_t *>(P.mlpm), 0u, np, ctx->st);  // +0.0f
  launch_fill_u32(reinterpret_cast<uint32_t *>(P.mlpv), 0u, np, ctx->st);
  for (int32_t t = 1; t <= steps; ++t) {
    launch_mlp_grad(hidden, w, rows, reinterpret_cast<const float4 *>(feat), target,
                    P.mlppart, P.mlpg, ctx->st);
    if (loss_out &&
        hipMemcpyAsync(&loss_out[t - 1], &P.mlpg[np], sizeof(float), hipMemcpyDeviceToHost,
                       ctx->st) != hipSuccess)
      return NBODY_EHIP;
    launch_adam(np, w, P.mlpg, P.mlpm, P.mlpv, t, lr, 0.9f, 0.999f, 1e-8f, ctx->st);
  }
  if ((s = hip_status()) != NBODY_OK) return s;
  if (hipStreamSynchronize(ctx->st) != hipSuccess) return NBODY_EHIP;
  return NBODY_OK;
}

nbody_status nbody_set_cost_model(nbody_ctx *ctx, int32_t hidden, const float *w) {
  nbody_status s = pre(ctx);
  if (s != NBODY_OK) return s;
  if (!w) {
    ctx->mlp_hidden = 0;
    return NBODY_OK;
  }
  if (!mlp_hidden_ok(hidden)) return NBODY_EINVAL;
  if (hipMemcpyAsync(ctx->P.mlpw, w, sizeof(float) * (size_t)mlp_nparams(hidden),
                     hipMemcpyDeviceToDevice, ctx->st) != hipSuccess)
    return NBODY_EHIP;
  ctx->mlp_hidden = hidden;
  return NBODY_OK;
}

nbody_status nbody_set_order(nbody_ctx *ctx, int32_t order) {
  if (!ctx) return NBODY_EINVAL;
  if (order < 0 || order > 3) return NBODY_EINVAL;
  ctx->order = order;
  return NBODY_OK;
}

nbody_status nbody_set_step_layout(nbody_ctx *ctx, int32_t layout) {
  if (!ctx) return NBODY_EINVAL;
  if (layout < 0 || layout > 2) return NBODY_EINVAL;
  ctx->step_layout = layout;
  return NBODY_OK;
}


nbody_status nbody_set_systems(nbody_ctx *ctx, int32_t n_sys, const int64_t *offsets) {
  nbody_status s = pre(ctx);
  if (s != NBODY_OK) return s;
  if (n_sys < 1 || n_sys > kMaxSystems || !offsets || offsets[0] != 0) return NBODY_EINVAL;
  for (int32_t i = 0; i < n_sys; ++i)
    if (offsets[i + 1] <= offsets[i]) return NBODY_EINVAL;  // every system non-empty
  if (offsets[n_sys] > ctx->L.n_max) return NBODY_ENOMEM;
  std::vector<uint32_t> off((size_t)n_sys + 1);
  for (int32_t i = 0; i <= n_sys; ++i) off[i] = (uint32_t)offsets[i];
  if (hipMemcpyAsync(ctx->P.sysoff, off.data(), sizeof(uint32_t) * off.size(),
                     hipMemcpyHostToDevice, ctx->st) != hipSuccess ||
      hipStreamSynchronize(ctx->st) != hipSuccess)
    return NBODY_EHIP;
  int r = 0;
  while (n_sys > 1 && (1 << (3 * r)) < n_sys) ++r;
  ctx->nsys = n_sys;
  ctx->sys_r = r;
  ctx->sys_n = offsets[n_sys];
  ctx->have_tree = false;
  return NBODY_OK;
}


}  // extern "C"

namespace {

// One global kick-drift-kick step (rebuild or refit), as nbody_step runs it.
nbody_status step_body(nbody_ctx *ctx, nbody_state *st, bool rebuild) {
  nbody_status s;
  const int64_t n = st->n;
  float *x32 = ctx->P.x32;
  const float hdt = (float)(0.5 * st->dt);
  launch_kick(n, st->vx, st->vy, st->vz, st->ax, st->ay, st->az, hdt, ctx->st);
  launch_drift(n, st->x, st->y, st->z, st->vx, st->vy, st->vz, st->dt, x32,
               drift_out(ctx, st, rebuild), ctx->st);
  if (rebuild) {
    if ((s = do_build(ctx, n, records(x32))) != NBODY_OK) return s;
  } else {
    if ((s = do_refit_sorted(ctx)) != NBODY_OK) return s;
  }
  ensure_asort(ctx, st);
  if ((s = do_calc(ctx, st->ax, st->ay, st->az, st->ax, st->ay, st->az)) != NBODY_OK)
    return s;
  launch_kick(n, st->vx, st->vy, st->vz, st->ax, st->ay, st->az, hdt, ctx->st);
  if (ctx->capturing) ctx->asort_src = nullptr;  // the next captured step mirrors afresh
  return hip_status();
}

nbody_ctx::GraphKey graph_key(const nbody_ctx *ctx, const nbody_state *st) {
  nbody_ctx::GraphKey k{};
  const void *p[10] = {st->x, st->y, st->z, st->vx, st->vy, st->vz, st->m, st->ax, st->ay, st->az};
  memcpy(k.p, p, sizeof(p));
  k.n = st->n;
  k.dt = st->dt;
  k.order = (ctx->order == 2 && ctx->mlp_hidden == 0) ? 0 : ctx->order;
  k.nsys = ctx->nsys;
  return k;
}

// Capture one step of `kind` (1: rebuild) on the private stream.
nbody_status capture_step(nbody_ctx *ctx, nbody_state *st, int kind) {
  hipStream_t orig = ctx->st;
  ctx->st = ctx->cap_st;
  ctx->capturing = true;
  nbody_status s = NBODY_OK;
  hipGraph_t g = nullptr;
  // a replay may follow changes to the state made between calls: every
  // captured step mirrors the accelerations afresh
  ctx->asort_src = nullptr;
  if (hipStreamBeginCapture(ctx->cap_st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    s = NBODY_EHIP;
  } else {
    s = step_body(ctx, st, kind == 1);
    if (hipStreamEndCapture(ctx->cap_st, &g) != hipSuccess && s == NBODY_OK) s = NBODY_EHIP;
  }
  ctx->capturing = false;
  ctx->st = orig;
  if (s != NBODY_OK) {
    if (g) (void)hipGraphDestroy(g);
    return s;
  }
  if (ctx->gexec[kind]) (void)hipGraphExecDestroy(ctx->gexec[kind]);
  ctx->gexec[kind] = nullptr;
  const hipError_t e = hipGraphInstantiate(&ctx->gexec[kind], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    ctx->gexec[kind] = nullptr;
    return NBODY_EHIP;
  }
  ctx->gkey[kind] = graph_key(ctx, st);
  return NBODY_OK;
}

}  // namespace

extern "C" {

nbody_status nbody_step_graph(nbody_ctx *ctx, nbody_state *st, int32_t n_steps) {
  nbody_status s = pre(ctx);
  if (s != NBODY_OK) return s;
  if (!st || st->level || st->rebuild_interval < 1 || st->integrator != kIntKDK)
    return NBODY_EINVAL;
  if (!ctx->cap_st) {
    if (hipStreamCreateWithFlags(&ctx->cap_st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->cap_ev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->cap_ev[1], hipEventDisableTiming) != hipSuccess)
      return NBODY_EHIP;
  }
  // argument checks and the first force evaluation, eagerly
  if ((s = nbody_step(ctx, st, 0)) != NBODY_OK) return s;
  if (n_steps == 0) return NBODY_OK;
  const nbody_ctx::GraphKey key = graph_key(ctx, st);
  if (hipEventRecord(ctx->cap_ev[0], ctx->st) != hipSuccess ||
      hipStreamWaitEvent(ctx->cap_st, ctx->cap_ev[0], 0) != hipSuccess)
    return NBODY_EHIP;
  for (int32_t k = 0; k < n_steps; ++k) {
    const int kind = (ctx->n != st->n || ctx->since_rebuild >= st->rebuild_interval) ? 1 : 0;
    if (!ctx->gexec[kind] || memcmp(&ctx->gkey[kind], &key, sizeof(key)) != 0)
      if ((s = capture_step(ctx, st, kind)) != NBODY_OK) return s;
    if (hipGraphLaunch(ctx->gexec[kind], ctx->cap_st) != hipSuccess) return NBODY_EHIP;
    if (kind == 1) {
      ctx->rebuilds++;
      ctx->since_rebuild = 0;
      ctx->n = st->n;
    }
    ctx->since_rebuild++;
    ctx->steps++;
    st->t += st->dt;
  }
  if (hipEventRecord(ctx->cap_ev[1], ctx->cap_st) != hipSuccess ||
      hipStreamWaitEvent(ctx->st, ctx->cap_ev[1], 0) != hipSuccess)
    return NBODY_EHIP;
  return hip_status();
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Tree forces on the library's own static scratch (no allocation by the call).
//
// The workspace of this entry point is the file-scope device array `scratch`.
// Host code never passes the array's name to a kernel (in host code it only
// stands in for the symbol); the device address comes from
// hipGetSymbolAddress, once per device, and is kept per device.
static constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kStaticMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kStaticMaxDevices] = {};

// The device address of `scratch` on device dev (the current device).
nbody_status static_scratch(int dev, void **out) {
  if (dev < 0 || dev >= kStaticMaxDevices) return NBODY_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return NBODY_EHIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return NBODY_OK;
}

__global__ void k_status_out(const DevScalars *sc, int32_t *out) { *out = sc->status; }
}  // namespace

extern "C" {

nbody_status nbody_tree_forces_noalloc(const nbody_params *p, void *hip_stream, int64_t n,
                                       const float *x, const float *y, const float *z,
                                       const float *m, const float *axo, const float *ayo,
                                       const float *azo, float *ax, float *ay, float *az,
                                       int32_t *status_dev) {
  nbody_status s = check_params(p);
  if (s != NBODY_OK) return s;
  if (n < 1 || !x || !y || !z || !m || !ax || !ay || !az) return NBODY_EINVAL;
  const int nnull = (axo == nullptr) + (ayo == nullptr) + (azo == nullptr);
  if (nnull != 0 && nnull != 3) return NBODY_EINVAL;
  int dev = 0;
  const int cu = device_cu_count(&dev);
  if (cu <= 0) return NBODY_EHIP;
  void *ws = nullptr;
  if ((s = static_scratch(dev, &ws)) != NBODY_OK) return s;
  // a small depth-first stack (groups that outgrow it go to the retry pass)
  // and no split walk keep the layout small; neither changes any result
  nbody_params q = *p;
  if (q.frontier_cap == 0 || q.frontier_cap > 256) q.frontier_cap = 256;
  q.walk_split = 1;
  q.order = 0;
  q.calcnode_sync = kCalcNodeLevels;
  const Layout L = make_layout(q, n, cu, false);
  if (L.total > kStaticScratchBytes) return NBODY_ENOMEM;
  nbody_ctx c;  // on the stack: no events, no pinned memory
  c.p = q;
  c.order = 0;
  c.st = static_cast<hipStream_t>(hip_stream);
  c.device = dev;
  c.num_cu = cu;
  c.ws = ws;
  c.ws_bytes = kStaticScratchBytes;
  c.L = L;
  c.P = carve(ws, L);
  c.bound = true;
  c.no_spans = true;
  if (!carve_complete(c.P, ws)) return NBODY_ECORRUPT;
  // the scratch keeps the previous call's contents: reset what starts at zero
  hipLaunchKernelGGL(k_scalars_init, dim3(1), dim3(1), 0, c.st, c.P.sc);
  if ((s = do_build(&c, n, Coords{x, y, z, m, 1})) != NBODY_OK) return s;
  if ((s = do_calc(&c, axo, ayo, azo, ax, ay, az)) != NBODY_OK) return s;
  if (status_dev) hipLaunchKernelGGL(k_status_out, dim3(1), dim3(1), 0, c.st, c.P.sc, status_dev);
  return hip_status();
}

}  // extern "C"
