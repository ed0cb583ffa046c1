// k_walk.hip -- group bounds and the group-wise tree walk (Sec. 1).
//
// One wavefront serves one i-group at a time, taking groups from a global
// work queue until the queue is empty (persistent kernel). For its group it
// traverses the tree from the root, depth first in chunks: the top 64 (or
// fewer) candidate cells of the wave's stack in global memory (the paper's
// per-SM cell buffer, Sec. 3) are popped and tested against the acceleration
// MAC of Eq. 2, one lane per cell; accepted cells enter the interaction list
// as pseudo-particles (centre of mass, mass), opened leaves contribute their
// particles, opened internal cells push their children (lane order). Each
// chunk pushes at most 512 cells, so the stack never holds more than 512 per
// tree level (under 11K cells), unlike a breadth-first frontier, which can
// hold a whole level. Offsets come from wave prefix sums. The list lives in
// LDS; whenever it holds `list_tile` entries it is flushed: every lane adds
// Eq. 1 over the tile for its particle, in FP32.
//
// Canonical order: list entries appear in the order of this traversal (a
// function of the tree and the group alone). Entry j belongs to block j / 64;
// each lane keeps four FP32 running sums and adds the entries of block b, in
// list order, to sum b mod 4; the four sums are added in that order at the
// end. A flush only cuts the sequence at block boundaries (tiles are
// multiples of 64 entries), so each lane's summation order is fixed by the
// group alone: it does not depend on the tile size, the stack capacity, the
// queue order, which wave runs the group, or the split below. Results are
// bit-identical across all of them. (The compensated sum keeps one running
// sum over the whole list and is never split.)
//
// Split walk: when few groups are queued (block steps often walk a few
// thousand heavy groups, fewer than the resident wavefronts), K = 2 or 4
// wavefronts take the same group: each traverses the whole tree (the MAC
// decisions are the same in each) but adds only the blocks b with
// b mod K == its part, i.e. the running sums r with r mod K == its part, and
// stores them; a second kernel (k_walk_join) adds the four sums per lane in
// order and writes the results. This turns a queue of q heavy groups into
// K q tasks of a quarter or half the arithmetic each.
//
// Lane layout: groups of at most 8, 16 or 32 members use S = 8, 4 or 2
// "streams": lane = stream * (64 / S) + member, stream s adds the entries
// whose list index is s mod S, and the S partial sums are combined at the
// end by a fixed butterfly. S depends only on the group size.
//
// Group-wise MAC (a reading of Eq. 2 for a shared list): d is the distance
// from the cell's centre of mass to the group's bounding box (no larger than
// any member's distance) and |a_old| the smallest previous acceleration in
// the group; accept iff d^2 > b^2 and delta_acc*|a_old|*d^4 >= G m b^2, all in
// FP32. Without a_old (bootstrap) accept iff d^2 > 4 b^2.
#include "nbody_internal.h"

namespace nb {

struct WalkArgs {
  const float4 *nodeA;
  const float4 *nodeB;
  const float4 *xyzm;
  const uint32_t *gbegin;
  const uint32_t *gcount;
  const float4 *gbox;
  const uint32_t *perm;
  const uint32_t *order;   // queue -> group (nullptr: identity)
  const uint32_t *qcount;  // queue length (device)
  const uint32_t *groot;   // per group root cell (nullptr: the root, cell 0)
  float4 *asort;           // key-ordered copy of the outputs with |a| (nullptr: none)
  uint32_t *retry;         // overflowing groups go here (nullptr: report instead)
  uint32_t *nretry;
  uint32_t *head;          // the work queue's claim counter
  uint32_t *frontier;
  uint32_t *gent;
  unsigned long long *ghash;
  DevScalars *sc;
  float *ax, *ay, *az;
  float *phi;              // potential output (the potential variant only)
  float *split;            // partial sums of split groups, per queue position
  float G, eps2;
  uint32_t n;
  uint32_t tile;
  uint32_t fmask;
  int bootstrap;
  int split_mode;          // -1 never (retry pass), 0 by queue length, else 1, 2, 4
  uint32_t split_slots;
};

// Wavefronts per group for a queue of ng groups walked by `waves` wavefronts.
__device__ __forceinline__ uint32_t split_factor(uint32_t ng, uint32_t waves, uint32_t slots,
                                                 int mode, bool comp) {
  if (comp || mode < 0 || ng > slots || ng > 4u * waves) return 1u;
  if (mode > 0) return (uint32_t)mode;
  return ng < 2u * waves ? 4u : ng < 4u * waves ? 2u : 1u;
}

__device__ __forceinline__ uint64_t mix64(uint64_t v) {
  v += 0x9E3779B97F4A7C15ull;
  v = (v ^ (v >> 30)) * 0xBF58476D1CE4E5B9ull;
  v = (v ^ (v >> 27)) * 0x94D049BB133111EBull;
  return v ^ (v >> 31);
}

// One lane's running sums of the acceleration components and, in the
// potential variant (kPot), of the potential: sum of -m_j / r_j.
template <bool kComp, bool kPot>
struct Acc3 {
  float x = 0.f, y = 0.f, z = 0.f, w = 0.f;
  __device__ __forceinline__ void add(float dx, float dy, float dz, float f, float mr) {
    x = __builtin_fmaf(f, dx, x);
    y = __builtin_fmaf(f, dy, y);
    z = __builtin_fmaf(f, dz, z);
    if constexpr (kPot) w = w - mr;
  }
  __device__ __forceinline__ void total(float &ox, float &oy, float &oz, float &ow) const {
    ox = x;
    oy = y;
    oz = z;
    ow = w;
  }
};

// Neumaier's compensated summation (Neumaier 1974) per component.
template <bool kPot>
struct Acc3<true, kPot> {
  float x = 0.f, y = 0.f, z = 0.f, w = 0.f, cx = 0.f, cy = 0.f, cz = 0.f, cw = 0.f;
  __device__ __forceinline__ static void nadd(float &s, float &c, float v) {
    const float t = s + v;
    c += (fabsf(s) >= fabsf(v)) ? ((s - t) + v) : ((v - t) + s);
    s = t;
  }
  __device__ __forceinline__ void add(float dx, float dy, float dz, float f, float mr) {
    nadd(x, cx, f * dx);
    nadd(y, cy, f * dy);
    nadd(z, cz, f * dz);
    if constexpr (kPot) nadd(w, cw, -mr);
  }
  __device__ __forceinline__ void total(float &ox, float &oy, float &oz, float &ow) const {
    ox = x + cx;
    oy = y + cy;
    oz = z + cz;
    ow = w + cw;
  }
};

// The running sums of a lane: four for the plain FP32 sum (block b of the
// list adds into sum b mod 4), one for the compensated sum. The sum of the
// block being added is always u0: after each block the sums rotate, so that
// no register is ever selected by a run-time index. A wavefront taking every
// K-th block (part p of K) holds the 4 / K sums p, p + K, ... in u0, u1, ...
// (rotating among those); after a whole number of rotation periods u_k holds
// sum p + K k.
constexpr uint32_t kBlk = 64;  // list entries per block
template <bool kComp, bool kPot>
struct RunSums;
template <bool kPot>
struct RunSums<false, kPot> {
  static constexpr uint32_t kNum = 4;
  Acc3<false, kPot> u0, u1, u2, u3;
  __device__ __forceinline__ void advance(uint32_t K) {
    if (K == 1u) {
      const Acc3<false, kPot> t = u0;
      u0 = u1;
      u1 = u2;
      u2 = u3;
      u3 = t;
    } else if (K == 2u) {
      const Acc3<false, kPot> t = u0;
      u0 = u1;
      u1 = t;
    }
  }
  __device__ __forceinline__ void total(float &ox, float &oy, float &oz, float &ow) const {
    ox = ((u0.x + u1.x) + u2.x) + u3.x;
    oy = ((u0.y + u1.y) + u2.y) + u3.y;
    oz = ((u0.z + u1.z) + u2.z) + u3.z;
    ow = ((u0.w + u1.w) + u2.w) + u3.w;
  }
};
template <bool kPot>
struct RunSums<true, kPot> {
  static constexpr uint32_t kNum = 1;
  Acc3<true, kPot> u0;
  __device__ __forceinline__ void advance(uint32_t) {}
  __device__ __forceinline__ void total(float &ox, float &oy, float &oz, float &ow) const {
    u0.total(ox, oy, oz, ow);
  }
};

// Entries of zero mass pad a flushed block to a multiple of S * kFlushUnroll,
// so every lane runs the same trip count and the loads of one trip are
// issued together. A padding entry adds exactly +0 to each sum (r^2 >= eps^2
// keeps it finite), and each lane still adds its entries in list order.
constexpr uint32_t kFlushUnroll = 4;
constexpr uint32_t kListPad = 8 * kFlushUnroll;  // largest S times the unroll

__device__ __forceinline__ void eq1_term(const float4 e, float4 pi, float eps2, float &dx,
                                         float &dy, float &dz, float &f, float &mr) {
  dx = e.x - pi.x;
  dy = e.y - pi.y;
  dz = e.z - pi.z;
  const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, eps2)));
  const float rinv = __builtin_amdgcn_rsqf(r2);
  mr = e.w * rinv;
  const float rinv2 = rinv * rinv;
  f = mr * rinv2;
}

// The stream count S is a template constant: the trip count and the LDS
// offsets of one trip (u * S entries past the trip's base) are then uniform
// and immediate.
template <bool kComp, bool kPot, uint32_t S>
__device__ __forceinline__ void flush_run_s(const float4 *__restrict__ list, uint32_t padded,
                                            uint32_t stream, float4 pi, float eps2,
                                            Acc3<kComp, kPot> &acc) {
  constexpr uint32_t step = S * kFlushUnroll;
  const float4 *p = list + stream;
  for (uint32_t j0 = 0; j0 < padded; j0 += step) {
    float4 e[kFlushUnroll];
#pragma unroll
    for (uint32_t u = 0; u < kFlushUnroll; ++u) e[u] = p[j0 + u * S];
#pragma unroll
    for (uint32_t u = 0; u < kFlushUnroll; ++u) {
      float dx, dy, dz, f, mr;
      eq1_term(e[u], pi, eps2, dx, dy, dz, f, mr);
      acc.add(dx, dy, dz, f, mr);
    }
  }
}

template <bool kComp, bool kPot>
__device__ __forceinline__ void flush_run(const float4 *__restrict__ list, uint32_t cnt,
                                          uint32_t stream, uint32_t S, float4 pi, float eps2,
                                          Acc3<kComp, kPot> &acc) {
  const uint32_t step = S * kFlushUnroll;
  const uint32_t padded = (cnt + step - 1) / step * step;
  // S is wave-uniform: these branches are not lane-predicated
  if (S == 1)
    flush_run_s<kComp, kPot, 1>(list, padded, stream, pi, eps2, acc);
  else if (S == 2)
    flush_run_s<kComp, kPot, 2>(list, padded, stream, pi, eps2, acc);
  else if (S == 4)
    flush_run_s<kComp, kPot, 4>(list, padded, stream, pi, eps2, acc);
  else
    flush_run_s<kComp, kPot, 8>(list, padded, stream, pi, eps2, acc);
}

// Flush the tile's cnt entries: whole blocks of 64 entries (the last one
// possibly short), each into u0 followed by a rotation of the sums (the
// compensated sum: all into its one sum). nblk counts the blocks added.
template <bool kComp, bool kPot>
__device__ __forceinline__ void flush_tile(float4 *__restrict__ list, uint32_t cnt, uint32_t K,
                                           uint32_t lane, uint32_t stream, uint32_t S,
                                           float4 pi, float eps2, RunSums<kComp, kPot> &R,
                                           uint32_t &nblk) {
  // every lane stores (two lanes per slot, same value): no lane-predicated
  // region; slots [cnt, cnt + kListPad) are free
  list[cnt + (lane & (kListPad - 1))] = make_float4(0.f, 0.f, 0.f, 0.f);
  __builtin_amdgcn_wave_barrier();
  if constexpr (kComp) {
    flush_run<kComp, kPot>(list, cnt, stream, S, pi, eps2, R.u0);
    return;
  }
  for (uint32_t off = 0; off < cnt; off += kBlk) {
    flush_run<kComp, kPot>(list + off, min(kBlk, cnt - off), stream, S, pi, eps2, R.u0);
    R.advance(K);
    ++nblk;
  }
}

// Per lane: the group member, the list stream, and (after adding the running
// sums) the butterfly over the streams; every lane ends with its member's sum.
__device__ __forceinline__ uint32_t stream_count(uint32_t gc) {
  return gc <= 8 ? 8u : gc <= 16 ? 4u : gc <= 32 ? 2u : 1u;
}

__device__ __forceinline__ void stream_reduce(uint32_t Wd, float &sx, float &sy, float &sz) {
  for (uint32_t d = Wd; d < 64u; d <<= 1) {
    sx += __shfl_xor(sx, (int)d, 64);
    sy += __shfl_xor(sy, (int)d, 64);
    sz += __shfl_xor(sz, (int)d, 64);
  }
}

__device__ __forceinline__ void stream_reduce1(uint32_t Wd, float &sw) {
  for (uint32_t d = Wd; d < 64u; d <<= 1) sw += __shfl_xor(sw, (int)d, 64);
}

// The results of member `lane` (< gc) of group (gb, gc): G times the sum, in
// caller order (in key order without perm), and with |a| into the
// key-ordered mirror when there is one.
__device__ __forceinline__ void store_group_result(const WalkArgs &a, uint32_t gb, uint32_t gc,
                                                   uint32_t lane, float sx, float sy,
                                                   float sz) {
  if (lane < gc) {  // lane == member here (stream 0)
    const uint32_t o = a.perm ? a.perm[gb + lane] : gb + lane;
    const float gx = a.G * sx, gy = a.G * sy, gz = a.G * sz;
    a.ax[o] = gx;
    a.ay[o] = gy;
    a.az[o] = gz;
    if (a.asort)
      a.asort[gb + lane] =
          make_float4(gx, gy, gz, sqrt_rn(__builtin_fmaf(gz, gz, __builtin_fmaf(gy, gy, gx * gx))));
  }
}

template <bool kComp, bool kHash, bool kPot>
__device__ __forceinline__ void walk_body(const WalkArgs &a, float4 *lds_list) {
  const uint32_t wv = threadIdx.x >> 6;
  const uint32_t lane = lane_id();
  // LDS: per wave a list tile, then per wave the chunk's owner table
  const uint32_t TS = a.tile + kListPad;  // tile + padding slots
  float4 *list = lds_list + wv * TS;
  float4 *s_ent = lds_list + kWalkWavesPerWG * TS + wv * 64;
  uint32_t *s_incl =
      reinterpret_cast<uint32_t *>(lds_list + kWalkWavesPerWG * (TS + 64)) + wv * 128;
  uint32_t *s_src = s_incl + 64;
  uint32_t *stk =
      a.frontier + (size_t)(blockIdx.x * kWalkWavesPerWG + wv) * (size_t)(a.fmask + 1);
  const uint32_t F = a.fmask + 1;
  const uint32_t ng = *a.qcount;
  const uint32_t ncell = a.sc->ncell;
  const uint32_t npart = a.n;
  // K wavefronts per group (a power of two); task t is part t mod K of
  // queue position t / K
  // (the compensated sum and the potential variant are never split)
  const uint32_t K = split_factor(ng, gridDim.x * kWalkWavesPerWG, a.split_slots, a.split_mode,
                                  kComp || kPot);
  const uint32_t kshift = K == 4u ? 2u : K == 2u ? 1u : 0u;
  // No lane-predicated region may sit in this loop: the compiler threads such
  // regions across the back-edge, and a wave that re-enters with lane 0 masked
  // off reads a stale queue index. Every lane joins the queue atomic (lane 0
  // adds 1, the rest 0) and the per-group results below are stored by every
  // lane (same value, same address).
  for (;;) {
    const uint32_t claim = atomicAdd(a.head, lane == 0 ? 1u : 0u);
    const uint32_t task = __builtin_amdgcn_readfirstlane(claim);
    const uint32_t qi = task >> kshift;
    const uint32_t part = task & (K - 1u);
    if (qi >= ng) break;
    const uint32_t g = a.order ? a.order[qi] : qi;
    const uint32_t gb = a.gbegin[g], gc = a.gcount[g];
    const float4 glo = a.gbox[2 * g], ghi = a.gbox[2 * g + 1];
    const float dA = glo.w;
    const uint32_t S = stream_count(gc);
    const uint32_t Wd = 64u / S;
    const uint32_t member = lane & (Wd - 1);
    const uint32_t stream = lane / Wd;
    const bool mem_ok = member < gc;
    const float4 pi = a.xyzm[gb + (mem_ok ? member : 0u)];
    RunSums<kComp, kPot> R;
    uint64_t hsum = 0;
    stk[0] = a.groot ? a.groot[g] : 0u;  // the walk's root (same value in every lane)
    uint32_t top = 1, visited = 0, cnt = 0;
    uint32_t entries = 0;  // list entries so far (list index of the next one)
    uint32_t nblk = 0;     // list blocks this wavefront has added
    bool overflow = false, corrupt = false;
    while (top > 0) {
      const uint32_t nc = min(64u, top);
      visited += nc;
      if (visited > ncell) {  // a tree visits each cell at most once
        corrupt = true;
        break;
      }
      top -= nc;
      const uint32_t cc = lane < nc ? stk[top + lane] : 0u;
      const bool bad_c = lane < nc && cc >= ncell;
      const bool has = lane < nc && !bad_c;
      const uint32_t c = has ? cc : 0u;
      float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = A;
      if (has) {
        A = a.nodeA[c];
        B = a.nodeB[c];
      }
      const uint32_t w0 = __float_as_uint(B.z), w1 = __float_as_uint(B.w);
      {
        const bool lf = (w1 & kLeafBit) != 0u;
        const uint32_t k = w1 & ~kLeafBit;
        const bool bad_n = has && (lf ? (w0 > npart || k > npart - w0)
                                      : (k > 8u || w0 > ncell || k > ncell - w0));
        if (__ballot(bad_c || bad_n)) {
          corrupt = true;
          break;
        }
      }
      bool accept = false;
      if (has) {
        const float tx = fmaxf(fmaxf(glo.x - A.x, A.x - ghi.x), 0.0f);
        const float ty = fmaxf(fmaxf(glo.y - A.y, A.y - ghi.y), 0.0f);
        const float tz = fmaxf(fmaxf(glo.z - A.z, A.z - ghi.z), 0.0f);
        const float d2 = __builtin_fmaf(tz, tz, __builtin_fmaf(ty, ty, tx * tx));
        if (d2 > A.w) {
          if (a.bootstrap) {
            const float four_b2 = 4.0f * A.w;
            accept = d2 > four_b2;
          } else {
            const float d4 = d2 * d2;
            const float lhs = dA * d4;
            accept = lhs >= B.y;
          }
        }
      }
      const bool leaf = (w1 & kLeafBit) != 0u;
      const uint32_t ne = !has ? 0u : accept ? 1u : leaf ? (w1 & ~kLeafBit) : 0u;
      const uint32_t nch = (has && !accept && !leaf) ? w1 : 0u;
      // children -> stack (over the popped chunk, in lane order) and entries
      // -> list: one scan of both counts (children <= 8 per lane, so at most
      // 512 per chunk: 10 bits; entries in the 22 bits above), or two scans
      // when a leaf is so large (coincident particles) that they might not fit
      uint32_t chi, chtot, ei, etot;
      if (__ballot(ne >= 65536u) == 0ull) {  // (wave-uniform)
        const uint32_t both = wave_incl_scan_dpp((ne << 10) | nch);
        const uint32_t btot = wave_last(both);
        chi = both & 1023u;
        chtot = btot & 1023u;
        ei = both >> 10;
        etot = btot >> 10;
      } else {
        chi = wave_incl_scan_dpp(nch);
        chtot = wave_last(chi);
        ei = wave_incl_scan_dpp(ne);
        etot = wave_last(ei);
      }
      if (top + chtot > F) {
        overflow = true;
        break;
      }
      // every lane has read its candidate before any lane overwrites it
      __builtin_amdgcn_wave_barrier();
      for (uint32_t k = 0; k < nch; ++k) stk[top + chi - nch + k] = w0 + k;
      top += chtot;
      // entries -> LDS list (flushing full tiles). Lane k owns entries
      // [incl_k - ne_k, incl_k); the copy is cooperative: lane r of the wave
      // fetches entry done + r, finding its owner by binary search. With
      // K > 1 only this part's blocks are copied.
      if (kHash) {
        if (accept) hsum += mix64((uint64_t)c);
        else if (ne)
          for (uint32_t k = 0; k < ne; ++k) hsum += mix64((1ull << 40) + w0 + k);
      }
      s_incl[lane] = ei;
      s_src[lane] = accept ? 0xffffffffu : w0;
      if (accept) s_ent[lane] = make_float4(A.x, A.y, A.z, B.x);
      __builtin_amdgcn_wave_barrier();
      uint32_t done = 0;
      while (done < etot) {
        const uint32_t J = entries + done;  // list index of the next entry
        uint32_t seg;
        if (K == 1u) {
          seg = min(a.tile - cnt, etot - done);
        } else {
          // the rest of block J / 64 within this chunk; the tile (a multiple
          // of 64 entries) holds whole blocks, so it always has room
          seg = min(kBlk - (J & (kBlk - 1u)), etot - done);
          if (((J / kBlk) & (K - 1u)) != part) {
            done += seg;
            continue;
          }
        }
        for (uint32_t r = lane; r < seg; r += 64u) {
          const uint32_t j = done + r;
          uint32_t k = 0;
#pragma unroll
          for (uint32_t s = 32; s >= 1; s >>= 1)
            if (s_incl[k + s - 1] <= j) k += s;
          const uint32_t src = s_src[k];
          const uint32_t first = k ? s_incl[k - 1] : 0u;
          list[cnt + r] = (src == 0xffffffffu) ? s_ent[k] : a.xyzm[src + (j - first)];
        }
        cnt += seg;
        done += seg;
        if (cnt == a.tile) {
          __builtin_amdgcn_wave_barrier();
          flush_tile<kComp, kPot>(list, cnt, K, lane, stream, S, pi, a.eps2, R, nblk);
          __builtin_amdgcn_wave_barrier();
          cnt = 0;
        }
      }
      __builtin_amdgcn_wave_barrier();  // owner table is rewritten next chunk
      entries += etot;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // overflow and corrupt are wave-uniform: these branches are not
    // lane-predicated; every lane joins the atomics and stores. Every part
    // of a split group meets the same overflow (same traversal); part 0
    // alone hands the group to the retry pass.
    const bool handoff = overflow && !corrupt && a.retry != nullptr;
    if (handoff) {
      if (part == 0u) {
        const uint32_t slot = __builtin_amdgcn_readfirstlane(
            atomicAdd(a.nretry, lane == 0 ? 1u : 0u));
        a.retry[slot] = g;
      }
    } else if (overflow || corrupt) {
      atomicOr(&a.sc->status, overflow ? kStOverflow : kStCorrupt);
    }
    if (overflow || corrupt) cnt = 0;
    __builtin_amdgcn_wave_barrier();
    flush_tile<kComp, kPot>(list, cnt, K, lane, stream, S, pi, a.eps2, R, nblk);
    __builtin_amdgcn_wave_barrier();
    // complete the rotation period (4 / K blocks): then u_k is sum part + K k
    if constexpr (!kComp)
      for (; nblk & (RunSums<kComp, kPot>::kNum / K - 1u); ++nblk) R.advance(K);
    if (K == 1u) {
      float sx, sy, sz, sw;
      R.total(sx, sy, sz, sw);
      stream_reduce(Wd, sx, sy, sz);
      store_group_result(a, gb, gc, lane, sx, sy, sz);
      if constexpr (kPot) {
        // the member's own entry (r = eps exactly) is in its list: add its
        // term back, phi_i = G (sum_j -m_j / r_j + m_i / eps)
        stream_reduce1(Wd, sw);
        if (lane < gc) {
          const float self = pi.w * __builtin_amdgcn_rsqf(a.eps2);
          a.phi[a.perm ? a.perm[gb + lane] : gb + lane] = a.G * (sw + self);
        }
      }
    } else if constexpr (!kComp && !kPot) {
      // this part's running sums into the queue slot: [sum][component][lane]
      float *slot = a.split + (size_t)qi * (kSplitSlotBytes / 4);
      slot[((part + 0u) * 3 + 0) * 64 + lane] = R.u0.x;
      slot[((part + 0u) * 3 + 1) * 64 + lane] = R.u0.y;
      slot[((part + 0u) * 3 + 2) * 64 + lane] = R.u0.z;
      if (K == 2u) {
        slot[((part + 2u) * 3 + 0) * 64 + lane] = R.u1.x;
        slot[((part + 2u) * 3 + 1) * 64 + lane] = R.u1.y;
        slot[((part + 2u) * 3 + 2) * 64 + lane] = R.u1.z;
      }
    }
    if (part == 0u) {
      if (kHash) {
        uint32_t lo = (uint32_t)hsum, hi = (uint32_t)(hsum >> 32);
        // 64-bit wave sum by 32-bit halves with carries
        for (int d = 32; d >= 1; d >>= 1) {
          const uint32_t olo = __shfl_xor(lo, d, 64), ohi = __shfl_xor(hi, d, 64);
          const uint32_t nlo = lo + olo;
          hi = hi + ohi + (nlo < lo ? 1u : 0u);
          lo = nlo;
        }
        a.ghash[g] = ((uint64_t)hi << 32) | lo;  // butterfly: every lane holds the sum
      }
      a.gent[g] = (overflow || corrupt) ? 0xffffffffu : entries;
    }
  }
}

// Second kernel of a split walk: per queue position, the four running sums
// of each lane added in order, then the stream butterfly and the results, as
// an unsplit walk ends. Groups the walk handed to its retry pass (entry
// count 0xffffffff) are left to it.
__global__ __launch_bounds__(256) void k_walk_join(WalkArgs a, uint32_t walk_waves) {
  const uint32_t ng = *a.qcount;
  if (split_factor(ng, walk_waves, a.split_slots, a.split_mode, false) == 1u) return;
  const uint32_t lane = lane_id();
  const uint32_t nw = gridDim.x * (blockDim.x >> 6);
  for (uint32_t qi = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) +
                                                    (threadIdx.x >> 6));
       qi < ng; qi += nw) {
    const uint32_t g = a.order ? a.order[qi] : qi;
    if (a.gent[g] == 0xffffffffu) continue;
    const uint32_t gb = a.gbegin[g], gc = a.gcount[g];
    const float *slot = a.split + (size_t)qi * (kSplitSlotBytes / 4);
    float v[4][3];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k) v[r][k] = slot[(r * 3 + k) * 64 + lane];
    float sx = ((v[0][0] + v[1][0]) + v[2][0]) + v[3][0];
    float sy = ((v[0][1] + v[1][1]) + v[2][1]) + v[3][1];
    float sz = ((v[0][2] + v[1][2]) + v[2][2]) + v[3][2];
    stream_reduce(64u / stream_count(gc), sx, sy, sz);
    store_group_result(a, gb, gc, lane, sx, sy, sz);
  }
}

// Interactions of the walked groups, and of those the tree's reference walk
// also took, now and then (the reference walk records them here): integer
// sums per workgroup into part[4 * blockIdx.x ..] (same-address atomics from
// every workgroup would serialise), added up by k_walk_stat_fold.
__global__ __launch_bounds__(256) void k_walk_stat(DevScalars *__restrict__ sc,
                                                   const uint32_t *__restrict__ order,
                                                   const uint32_t *__restrict__ gcount,
                                                   const uint32_t *__restrict__ gent,
                                                   uint32_t *__restrict__ gref, int record,
                                                   unsigned long long *__restrict__ part) {
  __shared__ unsigned long long s_sum[4][4];
  const uint32_t nq = order ? sc->nqueue : sc->ngroup;
  unsigned long long cur = 0, cur_a = 0, ref = 0, ent = 0;
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nq;
       q += gridDim.x * blockDim.x) {
    const uint32_t g = order ? order[q] : q;
    const uint32_t e = gent[g], c = gcount[g];
    if (e == 0xffffffffu) continue;
    const unsigned long long ec = (unsigned long long)e * c;
    cur += ec;
    ent += e;
    uint32_t r = gref[g];
    if (record && r == 0) {
      r = e;
      gref[g] = e;
    }
    if (r != 0) {
      cur_a += ec;
      ref += (unsigned long long)r * c;
    }
  }
  for (int d = 32; d >= 1; d >>= 1) {
    cur += __shfl_xor(cur, d, 64);
    cur_a += __shfl_xor(cur_a, d, 64);
    ref += __shfl_xor(ref, d, 64);
    ent += __shfl_xor(ent, d, 64);
  }
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) {
    s_sum[w][0] = cur;
    s_sum[w][1] = cur_a;
    s_sum[w][2] = ref;
    s_sum[w][3] = ent;
  }
  __syncthreads();
  if (threadIdx.x < 4)
    part[4 * blockIdx.x + threadIdx.x] = s_sum[0][threadIdx.x] + s_sum[1][threadIdx.x] +
                                         s_sum[2][threadIdx.x] + s_sum[3][threadIdx.x];
}

// The walk statistics: the partials' sums and the step's scalars (one
// workgroup of kStatBlocks threads).
__global__ __launch_bounds__(kStatBlocks) void k_walk_stat_fold(
    DevScalars *__restrict__ sc, const unsigned long long *__restrict__ part, int queued) {
  __shared__ unsigned long long s_sum[kStatBlocks / 64][4];
  unsigned long long v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = part[4 * threadIdx.x + k];
    for (int d = 32; d >= 1; d >>= 1) v[k] += __shfl_xor(v[k], d, 64);
  }
  if (lane_id() == 0)
    for (int k = 0; k < 4; ++k) s_sum[threadIdx.x >> 6][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t[4] = {0, 0, 0, 0};
    for (int w = 0; w < kStatBlocks / 64; ++w)
      for (int k = 0; k < 4; ++k) t[k] += s_sum[w][k];
    sc->wstat.ngroup = sc->ngroup;
    sc->wstat.queued = queued ? sc->nqueue : sc->ngroup;
    sc->wstat.inter = t[0];
    sc->wstat.inter_a = t[1];
    sc->wstat.inter_ref = t[2];
    sc->wstat.entries = t[3];
    sc->wstat.tick = sc->tick;
    sc->wstat.kmax = sc->kmax;
  }
}

// Both work queues' claim counters and the retry count start at zero.
__global__ void k_walk_prep(DevScalars *sc) {
  if (threadIdx.x == 0) {
    sc->queue_head = 0;
    sc->retry_head = 0;
    sc->nretry = 0;
  }
}

// The walk, and its retry pass as a kernel of its own (so that profiles and
// the walk timing see the main pass alone).
template <bool kComp, bool kHash>
__global__ __launch_bounds__(64 * kWalkWavesPerWG) void k_walk(WalkArgs a) {
  HIP_DYNAMIC_SHARED(float4, lds_list)
  walk_body<kComp, kHash, false>(a, lds_list);
}

template <bool kComp, bool kHash>
__global__ __launch_bounds__(64 * kWalkWavesPerWG) void k_walk_retry(WalkArgs a) {
  HIP_DYNAMIC_SHARED(float4, lds_list)
  walk_body<kComp, kHash, false>(a, lds_list);
}

// The potential variant (also writes phi; never split), main and retry pass.
template <bool kComp, bool kHash>
__global__ __launch_bounds__(64 * kWalkWavesPerWG) void k_walk_pot(WalkArgs a) {
  HIP_DYNAMIC_SHARED(float4, lds_list)
  walk_body<kComp, kHash, true>(a, lds_list);
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st) {
  int64_t g = cdiv(n, 256);
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_fill_u32, dim3(g), dim3(256), 0, st, p, v, n);
}

void launch_walk_stat(bool queued, bool record, const Ptrs &P, hipStream_t st) {
  hipLaunchKernelGGL(k_walk_stat, dim3(kStatBlocks), dim3(256), 0, st, P.sc,
                     queued ? P.order : nullptr, P.gcount, P.gent, P.gref, record ? 1 : 0,
                     P.wpart);
  hipLaunchKernelGGL(k_walk_stat_fold, dim3(1), dim3(kStatBlocks), 0, st, P.sc, P.wpart,
                     queued ? 1 : 0);
}


namespace {
WalkArgs walk_args(const WalkCfg &c, const uint32_t *perm, int64_t n, float *ax, float *ay,
                   float *az, const Ptrs &P) {
  WalkArgs a;
  a.nodeA = P.nodeA;
  a.nodeB = P.nodeB;
  a.xyzm = P.xyzm;
  a.gbegin = P.gbegin;
  a.gcount = P.gcount;
  a.gbox = P.gbox;
  a.perm = perm;
  a.order = c.use_order ? P.order : nullptr;
  a.qcount = c.use_order ? &P.sc->nqueue : &P.sc->ngroup;
  a.groot = c.batch ? P.groot : nullptr;
  a.asort = c.asort_out ? P.asort : nullptr;
  a.retry = P.retry;
  a.nretry = &P.sc->nretry;
  a.head = &P.sc->queue_head;
  a.frontier = P.frontier;
  a.gent = P.gent;
  a.ghash = P.ghash;
  a.sc = P.sc;
  a.ax = ax;
  a.ay = ay;
  a.az = az;
  a.phi = c.phi;
  a.G = c.G;
  a.eps2 = c.eps * c.eps;
  a.n = (uint32_t)n;
  a.tile = (uint32_t)c.list_tile;
  a.fmask = (uint32_t)c.frontier_cap - 1u;
  a.bootstrap = c.bootstrap;
  a.split = P.split;
  a.split_mode = c.split;
  a.split_slots = (uint32_t)c.split_slots;
  return a;
}

// per wave: list tile + padding (16 B/entry) + owner table (64 x (16 + 4 + 4) B)
size_t walk_lds(const WalkCfg &c) {
  return (size_t)kWalkWavesPerWG * ((c.list_tile + kListPad) * sizeof(float4) + 64 * 24);
}

}  // namespace

#define NB_WALK_LAUNCH(KERNEL, c, grid, lds, st, w)                           \
  do {                                                                         \
    const dim3 block_(64 * kWalkWavesPerWG);                                   \
    if ((c).compensated) {                                                     \
      if ((c).hash)                                                            \
        hipLaunchKernelGGL((KERNEL<true, true>), grid, block_, lds, st, w);    \
      else                                                                     \
        hipLaunchKernelGGL((KERNEL<true, false>), grid, block_, lds, st, w);   \
    } else {                                                                   \
      if ((c).hash)                                                            \
        hipLaunchKernelGGL((KERNEL<false, true>), grid, block_, lds, st, w);   \
      else                                                                     \
        hipLaunchKernelGGL((KERNEL<false, false>), grid, block_, lds, st, w);  \
    }                                                                          \
  } while (0)

void launch_walk(const WalkCfg &c, const uint32_t *perm, int64_t n, float *ax, float *ay,
                 float *az, const Ptrs &P, hipStream_t st) {
  const WalkArgs a = walk_args(c, perm, n, ax, ay, az, P);
  const int blocks = c.num_cu * c.waves_per_cu / kWalkWavesPerWG;
  hipLaunchKernelGGL(k_walk_prep, dim3(1), dim3(64), 0, st, P.sc);
  if (c.phi) {
    NB_WALK_LAUNCH(k_walk_pot, c, dim3(blocks), walk_lds(c), st, a);
    return;  // never split
  }
  NB_WALK_LAUNCH(k_walk, c, dim3(blocks), walk_lds(c), st, a);
  // a split walk's results (the kernel returns at once when the walk was not split)
  if (!c.compensated)
    hipLaunchKernelGGL(k_walk_join, dim3(512), dim3(256), 0, st, a,
                       (uint32_t)(blocks * kWalkWavesPerWG));
}

// Retry pass: the groups that outgrew a small stack (frontier_cap below the
// bound), walked by a few wavefronts whose stack holds 512 cells per level of
// the deepest tree; a second overflow is reported (it cannot happen).
void launch_walk_retry(const WalkCfg &c, const uint32_t *perm, int64_t n, float *ax,
                       float *ay, float *az, const Ptrs &P, hipStream_t st) {
  WalkArgs r = walk_args(c, perm, n, ax, ay, az, P);
  r.order = P.retry;
  r.qcount = &P.sc->nretry;
  r.retry = nullptr;
  r.frontier = P.frontier2;
  r.fmask = (uint32_t)c.frontier2_cap - 1u;
  r.head = &P.sc->retry_head;  // cleared with the walk's counters
  r.split_mode = -1;           // results written by the pass itself
  if (c.phi)
    NB_WALK_LAUNCH(k_walk_pot, c, dim3(c.retry_waves / kWalkWavesPerWG), walk_lds(c), st, r);
  else
    NB_WALK_LAUNCH(k_walk_retry, c, dim3(c.retry_waves / kWalkWavesPerWG), walk_lds(c), st, r);
}

}  // namespace nb
