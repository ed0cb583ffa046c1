// nbody_internal.h -- shared definitions of the gfx950 library (not public).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nbody.h"

namespace nb {

constexpr int kMaxLevel = 21;       // 3 x 21-bit Morton keys
constexpr int kLevels = kMaxLevel + 1;
constexpr uint32_t kLeafBit = 0x80000000u;  // node word w1: leaf flag
constexpr int kSortBits = 8;
constexpr int kSortRadix = 1 << kSortBits;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // keys per workgroup
constexpr int kBuildThreads = 256;                   // particles per build block
constexpr int kBuildHalo = 64;                       // >= max(leaf_max, group_max)
constexpr int kWalkWavesPerWG = 4;
constexpr int kStatBlocks = 256;  // workgroups of the walk statistics pass
// split walk: 4 partial sums x 3 components x 64 lanes (FP32) per queue position
constexpr int kSplitSlotBytes = 4 * 3 * 64 * 4;

// device status bits (sticky)
constexpr int32_t kStNonFinite = 1;
constexpr int32_t kStOverflow = 2;
constexpr int32_t kStCapacity = 4;
constexpr int32_t kStCorrupt = 8;  // internal consistency check failed

// Statistics of the last walk for the rebuild controller (copied to the host).
struct WalkStat {
  uint32_t ngroup, queued;
  unsigned long long inter;      // interactions of the walked groups
  unsigned long long inter_a;    // interactions of those walked groups that the
                                 // tree's first (reference) walk also took
  unsigned long long inter_ref;  // the same groups' interactions in that walk
  unsigned long long entries;    // list entries of the walked groups
  long long tick;                // block steps: the walk's step ends at this tick
  uint32_t kmax, pad;            // block steps: finest occupied level of that step
};

// Device scalars kept in the workspace.
struct DevScalars {
  uint32_t bbox[6];        // ordered-int min x,y,z then max x,y,z
  int32_t status;          // sticky error bits
  uint32_t ncell;
  uint32_t ngroup;
  uint32_t queue_head;     // walk work queue
  uint32_t lvl_off[kLevels + 1];
  double box[4];           // lo x,y,z and side L
  unsigned long long entries_total;
  unsigned long long inter_total;
  unsigned long long entries_acc;  // running totals while counting
  unsigned long long inter_acc;
  // individual block time steps (ticks of dt_max 2^-kTickBits)
  long long tick;          // current time
  long long tick0;         // start of the current step
  uint32_t kmax;           // finest occupied level during the current step
  uint32_t kmax_next;      // finest level after the closing kicks
  uint32_t nqueue;         // groups in the walk queue (order[])
  uint32_t nactive;        // particles active at the end of the current step
  uint32_t nretry;         // groups handed from the walk to its retry pass
  uint32_t retry_head;     // the retry pass's work queue
  uint32_t pad[2];
  WalkStat wstat;
  unsigned long long bar_epoch;  // launches of the grid-barrier calcNode so far
  uint32_t istart[kLevels + 1];  // internal cells of level l: ilist[istart[l] .. istart[l + 1])
  uint32_t nleaf;          // leaves of the current tree
  uint32_t pad2;
  // hashes of the caller's block-step state: [0] when a key-ordered call
  // scattered it back, [1] on entry to the next such call
  unsigned long long ko_hash[2];
};

// Offsets of the workspace, all 256-byte aligned.
struct Layout {
  int64_t n_max = 0;
  int64_t cell_cap = 0;
  int64_t sort_blocks = 0;
  int64_t build_blocks = 0;
  int64_t walk_waves = 0;
  int64_t frontier_cap = 0;
  int num_cu = 0;
  size_t off_lvlblk, off_bar;
  size_t off_scalars, off_keysA, off_keysB, off_valsA, off_valsB, off_hist,
      off_xyzm, off_x32, off_pinfo, off_leafof, off_blkcnt, off_clevel,
      off_cpbegin, off_cpcount, off_cfchild, off_cnchild, off_cparent,
      off_mom64, off_nodeA, off_nodeB, off_gbegin, off_gcount, off_gbox,
      off_gent, off_ghash, off_order, off_frontier, off_prevcnt, off_atmp, off_retry,
      off_frontier2, off_feat, off_target, off_pred, off_plast, off_okeys, off_qtmp, off_mlpw,
      off_mlpm, off_mlpv, off_mlpg, off_mlppart, off_gref, off_sysoff, off_sysbox, off_groot,
      off_inv, off_asort, off_split, off_gid, off_gflag, off_ilist, off_leaves, off_scan,
      off_longcnt, off_longslot, off_wpart;
  size_t off_kpos[2], off_kvel[2], off_kacc[2], off_kmass[2], off_kpt[2], off_klv[2];
  int64_t frontier2_cap = 0;  // retry pass stack: more than any tree needs
  int retry_waves = 0;
  int64_t split_slots = 0;  // queue positions with room for split-walk partial sums
  size_t total = 0;
};

struct Ptrs {
  DevScalars *sc;
  uint64_t *keysA, *keysB;
  uint32_t *valsA, *valsB;
  uint32_t *hist;       // sort histograms [radix][blocks] + totals[radix]
  float4 *xyzm;         // sorted x, y, z, m
  float *x32;           // FP32 (x, y, z, m) records of the state (caller order)
  uint32_t *pinfo;      // per sorted particle: s | D << 5 | (E + 1) << 10 | group start << 15
                        // (cells from level s to D start at it; its cells up to level E
                        // hold more than 64 particles)
  uint32_t *leafof;     // per sorted particle: its leaf cell
  uint32_t *blkcnt;     // scratch of block counts (build, groups, block-step queue)
  uint32_t *lvlblk;     // per level: cells starting in earlier build blocks [kLevels][blocks],
                        // then leaves [blocks] (+ totals), kept for the tree's life
  unsigned long long *bar;  // grid barrier flags: [kBarSlots] arrivals, [kBarSlots] releases
  int32_t *clevel;
  uint32_t *cpbegin, *cpcount;
  int32_t *cfchild, *cnchild, *cparent;
  double4 *mom64;       // M, Sx, Sy, Sz
  float4 *nodeA;        // com x, y, z, b2
  float4 *nodeB;        // m32, q, w0, w1 (bit patterns for w0/w1)
  uint32_t *gbegin, *gcount;
  float4 *gbox;         // [2g] = lo xyz, dA; [2g+1] = hi xyz, amin
  uint32_t *gent;       // per group: list entries of the last walk
  unsigned long long *ghash;
  uint32_t *order;      // walk queue order
  uint32_t *frontier;   // per wave ring
  uint32_t *prevcnt;    // per group: entries of the previous walk (ordering)
  float *atmp;          // [3][n] walk output of a block step (caller order)
  uint32_t *retry;      // groups whose frontier outgrew the main pass
  uint32_t *frontier2;  // retry pass frontier rings
  // cost model of the walk queue
  float4 *feat;         // per group: 4 features
  float *target;        // per group: log2 interactions of its last walk
  float *pred;          // per group: model prediction
  uint32_t *plast;      // per particle (caller order): list length of its last walk
  uint64_t *okeys;      // [2][n] queue sort keys
  uint32_t *qtmp;       // queue sort values before the digit pass
  float *mlpw;          // weights in use (largest model)
  float *mlpm, *mlpv, *mlpg;  // Adam moments, gradient + loss (training)
  float *mlppart;       // per-wavefront gradient shares
  uint32_t *gref;       // per group: list length in the tree's reference walk (0: none)
  uint32_t *sysoff;     // batch: system offsets [kMaxSystems + 1]
  double4 *sysbox;      // batch: per system root cube lo x, y, z, side L
  uint32_t *groot;      // batch: per group the walk's root cell
  uint32_t *inv;        // caller index -> sorted position of the current tree
  float4 *asort;        // key-ordered copy of the state's accelerations, |a| in w
  float *split;         // split walk: per queue position 4 x 3 x 64 partial sums
  uint32_t *gid;        // group of each sorted particle
  uint32_t *gflag;      // block steps: group holds a particle whose step ends (zero between steps)
  uint4 *ilist;         // internal cells in cell order, so level by level (istart):
                        // (cell, first child, children, particles)
  uint2 *leaves;        // leaves in particle order: (cell, first particle)
  uint32_t *scan;       // tile sums of the row scans
  uint32_t *longcnt;    // per build block: its cells longer than one block (<= kLevels)
  uint32_t *longslot;   // [blocks][kLevels] those cells
  unsigned long long *wpart;  // [kStatBlocks][4] partials of the walk statistics
  // block steps inside one nbody_step call: the state in key order, two sets
  // (a rebuild permutes set c into set 1 - c)
  double *kpos[2];      // [3][n] x, y, z (FP64)
  float *kvel[2];       // [3][n] vx, vy, vz
  float *kacc[2];       // [3][n] ax, ay, az of the last step
  float *kmass[2];      // [n]
  uint32_t *kpt[2];     // [n] caller index of each sorted slot
  int8_t *klv[2];       // [n] block-step levels
};

// stepping = false: no room for the key-ordered step state (tree forces only)
Layout make_layout(const nbody_params &p, int64_t n_max, int num_cu, bool stepping = true);
Ptrs carve(void *base, const Layout &L);

// FP32 coordinates and masses of particle i at x[i * stride], y[i * stride],
// ...: stride 1 for separate arrays, 4 for (x, y, z, m) records (x + 1 = y).
struct Coords {
  const float *x, *y, *z, *m;
  int64_t stride;
};

// ---- launchers (each enqueues on `st`; grid sizes depend only on n) ----
// part: 6 x ceil(n / 4096) words of scratch
void launch_bbox(const Coords &c, int64_t n, DevScalars *sc, uint32_t *part, hipStream_t st);
void launch_keys(const Coords &c, int64_t n, DevScalars *sc, uint64_t *keys, uint32_t *vals,
                 hipStream_t st);
// returns pointer (A or B) holding the sorted result
void launch_sort(int64_t n, uint64_t *keysA, uint32_t *valsA, uint64_t *keysB,
                 uint32_t *valsB, uint32_t *hist, hipStream_t st, uint64_t **keys_out,
                 uint32_t **vals_out);
void launch_gather(const Coords &c, const uint32_t *perm, int64_t n, float4 *xyzm,
                   hipStream_t st);
// r > 0: a batch of nsys systems (cells above level r always split, groups
// at level r or deeper, per-group walk roots in P.groot)
void launch_build(const uint64_t *keys, int64_t n, int leaf_max, int group_max,
                  int group_merge, int nsys, int r, const Ptrs &P, const Layout &L,
                  hipStream_t st);
// batch keys into P.keysA / P.valsA from P.sysoff; per-system cubes to P.sysbox
// (part: part_words words of scratch for partial bounds)
void launch_sys_keys(const Coords &c, int64_t n, int nsys, int r, const Ptrs &P,
                     uint32_t *part, int64_t part_words, hipStream_t st);
constexpr int kMaxSystems = 4096;
// calcNode synchronisation (nbody_params.calcnode_sync)
constexpr int kCalcNodeLevels = 1;  // one launch per tree level
constexpr int kCalcNodeGrid = 2;    // one persistent launch with a grid barrier
constexpr int kBarSlots = 1024;     // workgroups of the persistent launch, at most
// level_cells: internal cells per level of a recent tree (host array of
// kMaxLevel), or null; it only shapes the launches (levels with at most
// kNarrowCells cells are run by one workgroup), never the result
constexpr uint32_t kNarrowCells = 1024;
void launch_moments(int64_t n, float G, const Ptrs &P, const Layout &L, int mode,
                    const uint32_t *level_cells, hipStream_t st);
// asort (may be null): key-ordered a_old with |a|, read instead of a gather
// asort in a new key order from itself in the old one (inv_old: the old tree's
// caller index -> position; tmp: n float4 of scratch)
void launch_asort_remap(const uint32_t *perm, const uint32_t *inv_old, int64_t n,
                        float4 *asort, float4 *tmp, hipStream_t st);
void launch_asort_gather(const uint32_t *perm, int64_t n, const float *ax, const float *ay,
                         const float *az, float4 *asort, hipStream_t st);
// queued: the groups order[0 .. nqueue) only (block steps); else every group
void launch_group_bounds(const float *axo, const float *ayo, const float *azo,
                         const float4 *asort,
                         const uint32_t *perm, int64_t n, float delta_acc, bool queued,
                         const Ptrs &P, hipStream_t st);
struct WalkCfg {
  float G, eps;
  int bootstrap;
  int compensated;
  int list_tile;
  int frontier_cap;
  int waves_per_cu;
  int num_cu;
  int use_order;  // walk the groups order[0 .. nqueue) instead of all groups
  bool hash;      // record the per-group entry hash
  int64_t frontier2_cap;
  int retry_waves;
  bool batch;     // per-group roots (several systems in one tree)
  bool asort_out;  // also write the outputs, with |a|, to P.asort in key order
  int split;       // wavefronts per group: 0 by queue length, else 1, 2 or 4
  int64_t split_slots;
  float *phi = nullptr;  // potential output (caller order): the potential variant
};
// enqueue the walk kernel (after clearing its queue counters), then its
// retry pass for groups whose stack overflowed
void launch_walk(const WalkCfg &c, const uint32_t *perm, int64_t n, float *ax,
                 float *ay, float *az, const Ptrs &P, hipStream_t st);
void launch_walk_retry(const WalkCfg &c, const uint32_t *perm, int64_t n, float *ax,
                       float *ay, float *az, const Ptrs &P, hipStream_t st);
void launch_direct(int64_t n, const float *x, const float *y, const float *z,
                   const float *m, float G, float eps, float *ax, float *ay,
                   float *az, hipStream_t st);
void launch_direct64(int64_t n, const float *x, const float *y, const float *z,
                     const float *m, int64_t nt, const int64_t *tgt, double G, double eps,
                     double *ax, double *ay, double *az, double *aabs, double *phi,
                     hipStream_t st);
void launch_kick(int64_t n, float *vx, float *vy, float *vz, const float *ax,
                 const float *ay, const float *az, float hdt, hipStream_t st);
// Where a drift puts the FP32 image of the new positions: with xyzm set,
// straight into the key-ordered (x, y, z, m) array of the current tree
// through inv (caller index -> sorted position), which a refit then uses as
// is; otherwise into the (x, y, z, m) records x32 in caller order (for a rebuild).
struct SortedOut {
  float4 *xyzm;
  const uint32_t *inv;
  const float *m;
};
__device__ __forceinline__ void store_position(int64_t i, int64_t n, float fx, float fy,
                                               float fz, float *x32, const SortedOut &so) {
  (void)n;
  const float4 r = make_float4(fx, fy, fz, so.m[i]);
  if (so.xyzm)
    so.xyzm[so.inv ? so.inv[i] : (uint32_t)i] = r;  // no inv: the state is in key order
  else
    reinterpret_cast<float4 *>(x32)[i] = r;  // (x, y, z, m) records in caller order
}
void launch_drift(int64_t n, double *x, double *y, double *z, const float *vx,
                  const float *vy, const float *vz, double dt, float *x32, SortedOut so,
                  hipStream_t st);
// second-order Runge-Kutta (Heun): predict writes only the FP32 image of
// x + v dt; correct updates x, v from a and the predicted-position a_p
void launch_rk2_predict(int64_t n, const double *x, const double *y, const double *z,
                        const float *vx, const float *vy, const float *vz, double dt,
                        float *x32, SortedOut so, hipStream_t st);
void launch_rk2_correct(int64_t n, double *x, double *y, double *z, float *vx, float *vy,
                        float *vz, const float *ax, const float *ay, const float *az,
                        const float *apx, const float *apy, const float *apz, double dt,
                        float *x32, SortedOut so, hipStream_t st);
// inv[perm[s]] = s
void launch_invert(const uint32_t *perm, int64_t n, uint32_t *inv, hipStream_t st);

// Block-step calls of at least this many steps keep the state in key order
// (the gather on entry and the scatter on exit cost about what eight steps
// save).
constexpr int32_t kKeyedSteps = 8;

// One set of the key-ordered block-step state (slot s = sorted position).
struct KoSet {
  double *x, *y, *z;
  float *vx, *vy, *vz, *ax, *ay, *az, *m;
  uint32_t *pt;   // caller index of slot s
  int8_t *lv;
};
// Moves between caller order and key order go through 64-byte records, one
// per particle (x, y, z; vx, vy, vz; ax, ay, az; m; level; an index), held in
// the region of the key-ordered set that does not hold the state (each set's
// region is at least 64 n bytes): every particle then costs one random access
// of a whole record instead of eleven random 4- or 8-byte accesses.
// Caller order -> key order into set k: slot s takes caller index k.pt[s]
// (pt filled by the caller); rec = the other set's region. With skip (two
// hashes on the device), nothing is done when skip[0] == skip[1].
void launch_ko_gather(int64_t n, const KoSet &caller, const KoSet &k, uint4 *rec,
                      const unsigned long long *skip, hipStream_t st);
// *out = a 64-bit hash of the caller-order block-step state (positions,
// velocities, accelerations, masses, levels, by index; a sum of per-particle
// mixes, so any change of a value changes it except with probability about
// 2^-64). part: scratch of ko_hash_parts(n) words of 64 bits.
void launch_ko_hash(int64_t n, const double *x, const double *y, const double *z,
                    const float *vx, const float *vy, const float *vz, const float *ax,
                    const float *ay, const float *az, const float *m, const int8_t *level,
                    unsigned long long *out, unsigned long long *part, hipStream_t st);
int ko_hash_parts(int64_t n);
// Key order -> caller order from set k (positions, velocities, accelerations,
// levels; the caller's masses are not written); rec = the other set's
// region. Also writes inv[k.pt[s]] = s and, into *hash, the hash
// launch_ko_hash gives for the caller's arrays after the move (part: as
// there).
void launch_ko_scatter(int64_t n, const KoSet &k, const KoSet &caller, uint4 *rec,
                       uint32_t *inv, unsigned long long *hash, unsigned long long *part,
                       hipStream_t st);
// After a rebuild: slot s of the new order is slot perm[s] of the old one;
// with xyzm, also the tree's sorted (x, y, z, m) records, (float) of the FP64
// positions (what the drift stored as the records the keys came from).
void launch_ko_permute(int64_t n, const uint32_t *perm, const KoSet &from, const KoSet &to,
                       float4 *xyzm, hipStream_t st);
// Equal keys in caller order: the sort of a key-ordered state keeps equal
// keys in their old slot order; each run of equal keys is reordered by the
// caller index pt_old[vals[j]].
void launch_ko_ties(int64_t n, const uint64_t *keys, uint32_t *vals, const uint32_t *pt_old,
                    hipStream_t st);
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st);
// exclusive scan of rows[r][0 .. len) for r < nrows, row totals to totals[r];
// tsum: scan_scratch_words(len, nrows) words of scratch
void launch_scan_rows(uint32_t *rows, uint32_t len, int nrows, uint32_t *totals,
                      uint32_t *tsum, hipStream_t st);
int64_t scan_scratch_words(int64_t len, int nrows);

// sc->wstat of the walk just finished (queued: order[0 .. nqueue), else all)
// record: this walk is the tree's reference walk (its first with the
// acceleration criterion); it stores each walked group's list length in gref
void launch_walk_stat(bool queued, bool record, const Ptrs &P, hipStream_t st);

// single 8-bit digit pass of the stable radix sort (digit = key >> shift) of
// the first min(n, *n_dev) entries (n_dev may be null); n bounds the grid
void launch_digit_sort(int64_t n, const uint32_t *n_dev, int shift, const uint64_t *kin,
                       const uint32_t *vin, uint64_t *kout, uint32_t *vout, uint32_t *hist,
                       hipStream_t st);

// cost model of the walk queue
constexpr int kMlpMaxHidden = 64;
constexpr int kMlpMaxParams = 8 + 7 * kMlpMaxHidden + kMlpMaxHidden * kMlpMaxHidden + 1;
constexpr int kMlpWaves = 256;  // wavefronts of the gradient kernel
bool mlp_hidden_ok(int H);
int64_t mlp_nparams(int H);
void launch_mlp_forward(int H, const float *w, int64_t rows, const uint32_t *rows_dev,
                        const float4 *feat, float *y, hipStream_t st);
// grad_loss[0 .. np) = gradient of the mean squared error, grad_loss[np] = loss
void launch_mlp_grad(int H, const float *w, int64_t rows, const float4 *feat,
                     const float *target, float *partial, float *grad_loss, hipStream_t st);
void launch_adam(int64_t np, float *w, const float *g, float *m, float *v, int step, float lr,
                 float b1, float b2, float eps, hipStream_t st);
// w[0 .. 8): the model's input standardisation from the training rows
void launch_mlp_standardize(const float4 *feat, int64_t rows, float *w, hipStream_t st);
// features of the queued groups (queued) or of every group
void launch_cost_features(int64_t n, bool queued, const uint32_t *perm, const Ptrs &P,
                          hipStream_t st);
void launch_cost_after(int64_t n, bool queued, const uint32_t *perm, const Ptrs &P,
                       hipStream_t st);
// order[0 .. nqueue) by predicted cost (mode 1: count and previous list
// length, mode 2: the model); queued: sort the current queue, else all groups
void launch_cost_order(int64_t n, bool queued, int mode, int H, const Ptrs &P,
                       hipStream_t st);

// integrators (nbody_state.integrator)
constexpr int kIntKDK = 0;  // kick-drift-kick leapfrog
constexpr int kIntRK2 = 1;  // second-order Runge-Kutta, predict / correct

// individual block time steps
constexpr int kTickBits = 10;  // finest level: dt_max 2^-10
struct BlockCfg {
  double dt_max;
  double eta;
  float eps;
  int level_min, level_max;
};
void launch_blk_setup(long long tick, DevScalars *sc, hipStream_t st);
// level of every particle from a (at the current tick); kmax_next = max level
// part: scratch of 2 x (workgroups) words for the per-workgroup maxima and
// counts (the build's block counts, free outside a build)
void launch_blk_init(int64_t n, const float *ax, const float *ay, const float *az,
                     int8_t *level, const BlockCfg &c, DevScalars *sc, uint32_t *part,
                     hipStream_t st);
// kmax_next = max level; levels outside [level_min, level_max] set kStCorrupt
void launch_blk_scan(int64_t n, const int8_t *level, const BlockCfg &c, DevScalars *sc,
                     uint32_t *part, hipStream_t st);
// next tick; opening kicks at tick0; drift of every particle to tick
void launch_blk_begin(DevScalars *sc, hipStream_t st);
void launch_blk_open_drift(int64_t n, double *x, double *y, double *z, float *vx, float *vy,
                           float *vz, const float *ax, const float *ay, const float *az,
                           const int8_t *level, double dt_max, const DevScalars *sc,
                           float *x32, SortedOut so, hipStream_t st);
// walk queue = the groups holding a particle active at tick (group order)
void launch_blk_queue(int64_t n, const int8_t *level, const uint32_t *perm, const Ptrs &P,
                      hipStream_t st);
// active particles: a = anew (also into the key-ordered mirror asort through
// inv), closing kick, new level; kmax_next, nactive
void launch_blk_close(int64_t n, float *ax, float *ay, float *az, const float *nax,
                      const float *nay, const float *naz, float *vx, float *vy, float *vz,
                      int8_t *level, const BlockCfg &c, float4 *asort, const uint32_t *inv,
                      DevScalars *sc, uint32_t *part, hipStream_t st);
void launch_order_by_count(int64_t n, const Ptrs &P, hipStream_t st);

// ---- device helpers ----
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t l = __lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// wave-wide inclusive prefix sum of an unsigned value (all 64 lanes must be
// active; inactive contributions are passed as 0)
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t o = __shfl_up(v, d, 64);
    if ((int)__lane_id() >= d) v += o;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_bcast_last(uint32_t v) {
  return __shfl(v, 63, 64);
}

// Wave64 inclusive prefix sum with DPP (all 64 lanes active): prefix within
// each row of 16 lanes by row_shr 1, 2, 4, 8 (zero fill), then row 1 and 3
// add the last lane of the row before (row_bcast:15), rows 2 and 3 add lane
// 31 (row_bcast:31).
__device__ __forceinline__ uint32_t wave_incl_scan_dpp(uint32_t v) {
  int x = (int)v;
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false); // row_bcast:15
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false); // row_bcast:31
  return (uint32_t)x;
}

// value of lane 63, as a wave-uniform scalar
__device__ __forceinline__ uint32_t wave_last(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = fminf(v, __shfl_xor(v, d, 64));
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, 64));
  return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint32_t o = __shfl_xor(v, d, 64);
    v = o > v ? o : v;
  }
  return v;
}

// order-preserving float <-> uint map (for atomic min/max of floats)
__device__ __forceinline__ uint32_t f2ord(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Correctly rounded FP32 square root of a finite x >= 0. The hardware
// estimate (v_sqrt_f32, within about 1 ulp) is corrected by the midpoint
// test: y = RN(sqrt x) iff x lies between the squares of the midpoints to
// y's neighbours. A midpoint has at most 25 significant bits, so its square
// is exact in FP64, and sqrt(x) is never exactly a midpoint for an FP32 x.
__device__ __forceinline__ float sqrt_rn(float x) {
  float y = __builtin_sqrtf(x);
  if (!(x > 0.0f)) return y;  // 0 (and anything non-positive) as is
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const float yu = __uint_as_float(__float_as_uint(y) + 1u);
    const double mu = 0.5 * ((double)y + (double)yu);
    if ((double)x > mu * mu) {
      y = yu;
      continue;
    }
    const float yl = __uint_as_float(__float_as_uint(y) - 1u);
    const double ml = 0.5 * ((double)y + (double)yl);
    if ((double)x < ml * ml) {
      y = yl;
      continue;
    }
    break;
  }
  return y;
}

}  // namespace nb
