// k_moments.hip -- monopole moments of every cell ("calcNode", Sec. 2.2).
//
// M_J and S_J = sum m x are FP64: a leaf sums its particles sequentially in
// key order; an internal cell adds its children's unrounded sums in octant
// order. Stored once rounded: m32 = (float)M, com = (float)(S / M). The size
// b_J of Eq. 2 is read as the largest distance from com to a member
// particle: b2 = max over members of fmaf(dz,dz,fmaf(dy,dy,dx*dx)) with
// d = x - com in FP32; q = (G m32) b2 (FP32) is the left side of Eq. 2 times
// d^4. Levels are processed deepest first, one launch per level (the paper's
// calcNode likewise synchronises the whole grid once per level, App. A).
#include "nbody_internal.h"

namespace nb {

__device__ __forceinline__ float4 com_from(double M, double Sx, double Sy, double Sz,
                                           float4 first) {
  if (M > 0.0) return make_float4((float)(Sx / M), (float)(Sy / M), (float)(Sz / M), 0.f);
  return make_float4(first.x, first.y, first.z, 0.f);
}

__global__ __launch_bounds__(256) void k_mom_leaf(DevScalars *__restrict__ sc, uint32_t n,
                                                  const uint32_t *__restrict__ cpbegin,
                                                  const uint32_t *__restrict__ cpcount,
                                                  const int32_t *__restrict__ cnchild,
                                                  const float4 *__restrict__ xyzm,
                                                  double4 *__restrict__ mom64,
                                                  float4 *__restrict__ nodeA,
                                                  float4 *__restrict__ nodeB) {
  const uint32_t nc = sc->ncell;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc;
       c += (int64_t)gridDim.x * blockDim.x) {
    if (cnchild[c] != 0) continue;
    const uint32_t b = cpbegin[c], e = b + cpcount[c];
    if (b >= n || e > n || e <= b) {
      atomicOr(&sc->status, kStCorrupt);
      continue;
    }
    double mm = 0.0, xx = 0.0, yy = 0.0, zz = 0.0;
    for (uint32_t i = b; i < e; ++i) {
      const float4 p = xyzm[i];
      const double m = (double)p.w;
      mm += m;
      xx += m * (double)p.x;
      yy += m * (double)p.y;
      zz += m * (double)p.z;
    }
    const float4 com = com_from(mm, xx, yy, zz, xyzm[b]);
    float bb = 0.0f;
    for (uint32_t i = b; i < e; ++i) {
      const float4 p = xyzm[i];
      const float dx = p.x - com.x, dy = p.y - com.y, dz = p.z - com.z;
      const float d2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
      bb = d2 > bb ? d2 : bb;
    }
    mom64[c] = make_double4(mm, xx, yy, zz);
    nodeA[c] = make_float4(com.x, com.y, com.z, bb);
    nodeB[c].x = (float)mm;
  }
}

__global__ __launch_bounds__(256) void k_mom_level(DevScalars *__restrict__ sc,
                                                   int level,
                                                   const uint32_t *__restrict__ cpbegin,
                                                   const int32_t *__restrict__ cfchild,
                                                   const int32_t *__restrict__ cnchild,
                                                   const float4 *__restrict__ xyzm,
                                                   double4 *__restrict__ mom64,
                                                   float4 *__restrict__ nodeA,
                                                   float4 *__restrict__ nodeB) {
  if (sc->ncell == 0) return;
  const uint32_t c0 = sc->lvl_off[level], c1 = sc->lvl_off[level + 1];
  for (int64_t c = c0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < c1;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int k = cnchild[c];
    if (k == 0) continue;
    const int32_t f = cfchild[c];
    if (f <= (int32_t)c || k > 8 || (uint32_t)(f + k) > sc->ncell) {
      atomicOr(&sc->status, kStCorrupt);
      continue;
    }
    double mm = 0.0, xx = 0.0, yy = 0.0, zz = 0.0;
    for (int q = 0; q < k; ++q) {
      const double4 s = mom64[f + q];
      mm += s.x;
      xx += s.y;
      yy += s.z;
      zz += s.w;
    }
    const float4 com = com_from(mm, xx, yy, zz, xyzm[cpbegin[c]]);
    mom64[c] = make_double4(mm, xx, yy, zz);
    nodeA[c] = make_float4(com.x, com.y, com.z, 0.0f);  // b2 set by k_mom_b2
    nodeB[c].x = (float)mm;
  }
}

// b2 of internal cells: every particle visits its ancestors (leaf excluded)
// level by level; lanes of one block that share a cell reduce in LDS first,
// then one atomic max per (block, cell) on the bit pattern (b2 >= 0, so the
// float order equals the unsigned order).
__global__ __launch_bounds__(256) void k_mom_b2(DevScalars *__restrict__ sc, uint32_t n,
                                                const uint32_t *__restrict__ pinfo,
                                                const uint32_t *__restrict__ leafof,
                                                const int32_t *__restrict__ cparent,
                                                const float4 *__restrict__ xyzm,
                                                float4 *__restrict__ nodeA) {
  __shared__ uint32_t slot[256];
  __shared__ uint32_t red[3][4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool valid = i < n;
  slot[threadIdx.x] = 0u;
  float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
  int lvl = -1;
  int32_t cur = -1;
  if (valid) {
    p = xyzm[i];
    const int D = (pinfo[i] >> 5) & 31;
    const uint32_t lf = leafof[i];
    if (D > 0 && lf < sc->ncell) {
      cur = cparent[lf];
      lvl = D - 1;
    }
  }
  const int w = threadIdx.x >> 6;
  // highest starting level in the block
  {
    const uint32_t m = wave_max_u32((uint32_t)(lvl + 1));
    if (lane_id() == 0) red[0][w] = m;
  }
  __syncthreads();
  int top = (int)max(max(red[0][0], red[0][1]), max(red[0][2], red[0][3])) - 1;
  __syncthreads();
  for (int l = top; l >= 0; --l) {
    bool act = valid && lvl == l;
    // range of active cells in the block
    uint32_t cmin = act ? (uint32_t)cur : 0xffffffffu;
    uint32_t cmax = act ? (uint32_t)cur : 0u;
    {
      uint32_t a = cmin, b = cmax;
#pragma unroll
      for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t oa = __shfl_xor(a, d, 64), ob = __shfl_xor(b, d, 64);
        a = oa < a ? oa : a;
        b = ob > b ? ob : b;
      }
      if (lane_id() == 0) {
        red[1][w] = a;
        red[2][w] = b;
      }
    }
    __syncthreads();
    uint32_t bmin = red[1][0], bmax = red[2][0];
    for (int q = 1; q < 4; ++q) {
      bmin = red[1][q] < bmin ? red[1][q] : bmin;
      bmax = red[2][q] > bmax ? red[2][q] : bmax;
    }
    uint32_t d2bits = 0u;
    if (act && (cur < 0 || (uint32_t)cur >= sc->ncell)) {
      atomicOr(&sc->status, kStCorrupt);
      act = false;
    }
    if (act) {
      const float4 c = nodeA[cur];
      const float dx = p.x - c.x, dy = p.y - c.y, dz = p.z - c.z;
      d2bits = __float_as_uint(__builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx)));
    }
    // whole wave on one cell: reduce in registers first
    const uint64_t am = __ballot(act);
    const int32_t c0 = __shfl(cur, (int)(am ? __builtin_ctzll(am) : 0), 64);
    const bool same = am != 0 && __ballot(act && cur == c0) == am;
    if (same) {
      const uint32_t m = wave_max_u32(d2bits);
      if (lane_id() == (uint32_t)__builtin_ctzll(am) && (uint32_t)cur - bmin < 256u)
        atomicMax(&slot[(uint32_t)cur - bmin], m);
    } else if (act && (uint32_t)cur - bmin < 256u) {
      atomicMax(&slot[(uint32_t)cur - bmin], d2bits);
    }
    __syncthreads();
    if (bmin != 0xffffffffu && threadIdx.x <= bmax - bmin && bmin + threadIdx.x < sc->ncell) {
      const uint32_t v = slot[threadIdx.x];
      const uint32_t c = bmin + threadIdx.x;
      if (v > __float_as_uint(nodeA[c].w))
        atomicMax(reinterpret_cast<uint32_t *>(&nodeA[c].w), v);
      slot[threadIdx.x] = 0u;
    }
    __syncthreads();
    if (act) {
      cur = cparent[cur];
      lvl = l - 1;
      if (l > 0 && (cur < 0 || (uint32_t)cur >= sc->ncell)) {
        atomicOr(&sc->status, kStCorrupt);
        lvl = -1;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_mom_final(const DevScalars *__restrict__ sc,
                                                   float G,
                                                   const float4 *__restrict__ nodeA,
                                                   float4 *__restrict__ nodeB) {
  const uint32_t nc = sc->ncell;
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < nc;
       c += (int64_t)gridDim.x * blockDim.x) {
    const float gm = G * nodeB[c].x;
    nodeB[c].y = gm * nodeA[c].w;
  }
}

void launch_moments(int64_t n, float G, const Ptrs &P, const Layout &L, hipStream_t st) {
  int64_t gc = cdiv(L.cell_cap, 256);
  if (gc > 4096) gc = 4096;
  if (gc < 1) gc = 1;
  hipLaunchKernelGGL(k_mom_leaf, dim3(gc), dim3(256), 0, st, P.sc, (uint32_t)n, P.cpbegin, P.cpcount,
                     P.cnchild, P.xyzm, P.mom64, P.nodeA, P.nodeB);
  int64_t gl = cdiv(n, 256 * 4);
  if (gl > 2048) gl = 2048;
  if (gl < 1) gl = 1;
  for (int l = kMaxLevel - 1; l >= 0; --l)
    hipLaunchKernelGGL(k_mom_level, dim3(gl), dim3(256), 0, st, P.sc, l, P.cpbegin,
                       P.cfchild, P.cnchild, P.xyzm, P.mom64, P.nodeA, P.nodeB);
  hipLaunchKernelGGL(k_mom_b2, dim3(cdiv(n, 256)), dim3(256), 0, st, P.sc, (uint32_t)n,
                     P.pinfo, P.leafof, P.cparent, P.xyzm, P.nodeA);
  hipLaunchKernelGGL(k_mom_final, dim3(gc), dim3(256), 0, st, P.sc, G, P.nodeA, P.nodeB);
}

}  // namespace nb
