// k_keys.hip -- root cube, 63-bit Morton keys and the key-order gather.
//
// The paper builds its tree from sorted particles ("makeTree", Sec. 2.2 and
// Sec. 4.1) without naming the key. Here: the root cube has its corner at
// the exact FP32 minimum of each axis and side L = the smallest power of two
// not below the largest axis extent (computed in FP64); each axis is
// quantised to 21 bits, q = min(floor((x - lo) * 2^21 / L), 2^21 - 1), and
// the bits are interleaved x, y, z from the most significant end, so the
// level-l octant digit is bits 3(21-l)..3(21-l)+2 of the key.
#include "nbody_internal.h"

namespace nb {

// Bounds of the particles: each workgroup reduces its share to six ordered
// integers in part[6 * block] (min x, y, z, max x, y, z); k_bbox_fold
// reduces the blocks (no atomics on the six words: thousands of workgroups
// contending for them were most of the pass).
__global__ __launch_bounds__(256) void k_bbox(Coords c, int64_t n, DevScalars *sc,
                                              uint32_t *__restrict__ part) {
  float lo[3] = {INFINITY, INFINITY, INFINITY};
  float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  auto take = [&](float x, float y, float z) {
    const float v[3] = {x, y, z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      bad |= !isfinite(v[k]);
      lo[k] = fminf(lo[k], v[k]);
      hi[k] = fmaxf(hi[k], v[k]);
    }
  };
  // kU particles per trip, their loads issued together; (x, y, z, m)
  // records are read as one 16-byte load each
  constexpr int kU = 8;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const bool rec = c.stride == 4;
  for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i0 < n; i0 += kU * stride) {
    float4 q[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t i = i0 + u * stride;
      const int64_t j = i < n ? i : i0;  // (i0 < n)
      q[u] = rec ? reinterpret_cast<const float4 *>(c.x)[j]
                 : make_float4(c.x[j], c.y[j], c.z[j], 0.0f);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (i0 + u * stride < n) take(q[u].x, q[u].y, q[u].z);
  }
  __shared__ float red[6][4];
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float a = wave_min(lo[k]);
    const float b = wave_max(hi[k]);
    if (lane_id() == 0) {
      red[k][w] = a;
      red[3 + k][w] = b;
    }
  }
  if (__any(bad) && lane_id() == 0) atomicOr(&sc->status, kStNonFinite);
  __syncthreads();
  if (threadIdx.x < 3) {
    const int k = threadIdx.x;
    float a = red[k][0], b = red[3 + k][0];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) {
      a = fminf(a, red[k][q]);
      b = fmaxf(b, red[3 + k][q]);
    }
    part[6 * blockIdx.x + k] = f2ord(a);
    part[6 * blockIdx.x + 3 + k] = f2ord(b);
  }
}

__global__ __launch_bounds__(256) void k_bbox_fold(const uint32_t *__restrict__ part, int nb,
                                                   DevScalars *sc) {
  uint32_t lo[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, hi[3] = {0u, 0u, 0u};
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      lo[k] = min(lo[k], part[6 * b + k]);
      hi[k] = max(hi[k], part[6 * b + 3 + k]);
    }
  __shared__ uint32_t red[6][4];
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    uint32_t a = lo[k], c = hi[k];
    for (int d = 32; d >= 1; d >>= 1) {
      a = min(a, (uint32_t)__shfl_xor((int)a, d, 64));
      c = max(c, (uint32_t)__shfl_xor((int)c, d, 64));
    }
    if (lane_id() == 0) {
      red[k][w] = a;
      red[3 + k][w] = c;
    }
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int k = threadIdx.x;
    uint32_t a = red[k][0], c = red[3 + k][0];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) {
      a = min(a, red[k][q]);
      c = max(c, red[3 + k][q]);
    }
    sc->bbox[k] = a;
    sc->bbox[3 + k] = c;
  }
}

// Spread the low 21 bits of v so that bit b lands on bit 3b.
__device__ __forceinline__ uint64_t spread3(uint32_t v) {
  uint64_t x = v & 0x1fffffu;
  x = (x | (x << 32)) & 0x001f00000000ffffull;
  x = (x | (x << 16)) & 0x001f0000ff0000ffull;
  x = (x | (x << 8)) & 0x100f00f00f00f00full;
  x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
  x = (x | (x << 2)) & 0x1249249249249249ull;
  return x;
}

__device__ __forceinline__ uint32_t quantise21(float v, double lo, double scale) {
  const double t = ((double)v - lo) * scale;
  if (t >= 2097151.0) return 2097151u;
  if (t <= 0.0) return 0u;
  return (uint32_t)t;  // t > 0: truncation is floor
}

__global__ __launch_bounds__(256) void k_keys(Coords c,
                                              int64_t n, DevScalars *sc,
                                              uint64_t *__restrict__ keys,
                                              uint32_t *__restrict__ vals) {
  // root cube from the reduced bounds (every thread recomputes it)
  double lo[3], ext = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float a = ord2f(sc->bbox[k]);
    const float b = ord2f(sc->bbox[3 + k]);
    lo[k] = (double)a;
    const double e = (double)b - (double)a;
    ext = e > ext ? e : ext;
  }
  int eL = 0;  // L = 2^eL
  if (ext > 0.0) {
    int e;
    const double f = frexp(ext, &e);
    eL = (f == 0.5) ? e - 1 : e;
  }
  const double scale = ldexp(1.0, 21 - eL);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->box[0] = lo[0];
    sc->box[1] = lo[1];
    sc->box[2] = lo[2];
    sc->box[3] = ldexp(1.0, eL);
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t qx = quantise21(c.x[i * c.stride], lo[0], scale);
    const uint32_t qy = quantise21(c.y[i * c.stride], lo[1], scale);
    const uint32_t qz = quantise21(c.z[i * c.stride], lo[2], scale);
    keys[i] = (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
    vals[i] = (uint32_t)i;
  }
}

// ---- several independent systems in one tree (system s holds caller
// indices [off[s], off[s+1])): each system gets its own root cube, and its
// index fills the top r octal digits of the key above a (21 - r)-level
// Morton key in that cube.

// lo and L of a system's root cube from the exact bounds (p: minima, q:
// maxima) of its particles.
__device__ __forceinline__ double4 sys_cube(const float p[3], const float q[3]) {
  double l[3], ext = 0.0;
  for (int k = 0; k < 3; ++k) {
    l[k] = (double)p[k];
    const double e = (double)q[k] - (double)p[k];
    ext = e > ext ? e : ext;
  }
  int eL = 0;
  if (ext > 0.0) {
    int e;
    const double f = frexp(ext, &e);
    eL = (f == 0.5) ? e - 1 : e;
  }
  return make_double4(l[0], l[1], l[2], ldexp(1.0, eL));
}

// Exact bounds of share k = blockIdx.y of gridDim.y consecutive shares of
// system s = blockIdx.x. With one share per system the workgroup writes the
// system's root cube itself; otherwise it writes its bounds to
// part[6 * (s * shares + k) ..] (min x, y, z, max x, y, z) and
// k_sys_bbox_fold reduces them (one workgroup for a system of 2^18 particles
// was most of the batch's key pass).
__global__ __launch_bounds__(256) void k_sys_bbox(Coords c,
                                                  const uint32_t *__restrict__ off,
                                                  double4 *__restrict__ sysbox,
                                                  DevScalars *sc, float *__restrict__ part) {
  const uint32_t s = blockIdx.x, k = blockIdx.y, shares = gridDim.y;
  const uint32_t a0 = off[s], len = off[s + 1] - a0;
  const uint32_t per = (uint32_t)(((uint64_t)len + shares - 1) / shares);
  const uint32_t a = a0 + (uint32_t)std::min<uint64_t>(len, (uint64_t)k * per);
  const uint32_t b = a0 + (uint32_t)std::min<uint64_t>(len, (uint64_t)(k + 1) * per);
  float lo[3] = {INFINITY, INFINITY, INFINITY};
  float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  for (uint32_t i = a + threadIdx.x; i < b; i += blockDim.x) {
    const float v[3] = {c.x[i * c.stride], c.y[i * c.stride], c.z[i * c.stride]};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      bad |= !isfinite(v[k]);
      lo[k] = fminf(lo[k], v[k]);
      hi[k] = fmaxf(hi[k], v[k]);
    }
  }
  __shared__ float red[6][4];
  const int w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float p = wave_min(lo[k]);
    const float q = wave_max(hi[k]);
    if (lane_id() == 0) {
      red[k][w] = p;
      red[3 + k][w] = q;
    }
  }
  if (__any(bad) && lane_id() == 0) atomicOr(&sc->status, kStNonFinite);
  __syncthreads();
  if (threadIdx.x == 0) {
    float p[3], q[3];
    for (int k = 0; k < 3; ++k) {
      p[k] = red[k][0];
      q[k] = red[3 + k][0];
      for (int j = 1; j < (int)(blockDim.x >> 6); ++j) {
        p[k] = fminf(p[k], red[k][j]);
        q[k] = fmaxf(q[k], red[3 + k][j]);
      }
    }
    if (shares == 1) {
      sysbox[s] = sys_cube(p, q);
    } else {
      float *o = part + 6 * ((size_t)s * shares + k);
      for (int j = 0; j < 3; ++j) {
        o[j] = p[j];
        o[3 + j] = q[j];
      }
    }
  }
}

// One thread per system: the shares' bounds, then its root cube.
__global__ __launch_bounds__(256) void k_sys_bbox_fold(const float *__restrict__ part,
                                                       int shares, int nsys,
                                                       double4 *__restrict__ sysbox) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsys) return;
  float p[3] = {INFINITY, INFINITY, INFINITY}, q[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int k = 0; k < shares; ++k) {
    const float *o = part + 6 * ((size_t)s * shares + k);
    for (int j = 0; j < 3; ++j) {
      p[j] = fminf(p[j], o[j]);
      q[j] = fmaxf(q[j], o[3 + j]);
    }
  }
  sysbox[s] = sys_cube(p, q);
}

__device__ __forceinline__ uint32_t quantise_bits(float v, double lo, double scale,
                                                  double top) {
  const double t = ((double)v - lo) * scale;
  if (t >= top) return (uint32_t)top;
  if (t <= 0.0) return 0u;
  return (uint32_t)t;
}

__global__ __launch_bounds__(256) void k_sys_keys(Coords c, int64_t n,
                                                  const uint32_t *__restrict__ off, int nsys,
                                                  int r, const double4 *__restrict__ sysbox,
                                                  uint64_t *__restrict__ keys,
                                                  uint32_t *__restrict__ vals) {
  const int bits = kMaxLevel - r;
  const double top = ldexp(1.0, bits) - 1.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    // system of i: the last s with off[s] <= i
    int lo = 0, hi = nsys;  // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (off[mid] <= (uint32_t)i)
        lo = mid;
      else
        hi = mid;
    }
    const double4 bx = sysbox[lo];
    const double scale = ldexp(1.0, bits) / bx.w;
    const uint32_t qx = quantise_bits(c.x[i * c.stride], bx.x, scale, top);
    const uint32_t qy = quantise_bits(c.y[i * c.stride], bx.y, scale, top);
    const uint32_t qz = quantise_bits(c.z[i * c.stride], bx.z, scale, top);
    keys[i] = ((uint64_t)lo << (3 * bits)) | (spread3(qx) << 2) | (spread3(qy) << 1) |
              spread3(qz);
    vals[i] = (uint32_t)i;
  }
}

__global__ __launch_bounds__(256) void k_invert(const uint32_t *__restrict__ perm, int64_t n,
                                                uint32_t *__restrict__ inv) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n;
       s += (int64_t)gridDim.x * blockDim.x)
    inv[perm[s]] = (uint32_t)s;
}

__global__ __launch_bounds__(256) void k_gather(Coords c,
                                                const uint32_t *__restrict__ perm,
                                                int64_t n, float4 *__restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t p = perm[i];
    out[i] = c.stride == 4 ? reinterpret_cast<const float4 *>(c.x)[p]
                           : make_float4(c.x[p], c.y[p], c.z[p], c.m[p]);
  }
}

static int grid_for(int64_t n, int per_thread, int cap) {
  int64_t g = cdiv(n, 256LL * per_thread);
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

void launch_bbox(const Coords &c, int64_t n, DevScalars *sc, uint32_t *part, hipStream_t st) {
  const int nb = grid_for(n, 16, 1024);  // 6 words of part per block
  hipLaunchKernelGGL(k_bbox, dim3(nb), dim3(256), 0, st, c, n, sc, part);
  hipLaunchKernelGGL(k_bbox_fold, dim3(1), dim3(256), 0, st, part, nb, sc);
}

void launch_sys_keys(const Coords &c, int64_t n, int nsys, int r, const Ptrs &P,
                     uint32_t *part, int64_t part_words, hipStream_t st) {
  // shares per system: up to 32 (2048 workgroups for 64 systems), as the
  // scratch allows; a single share writes the cube directly
  const int shares = (int)std::max<int64_t>(
      1, std::min<int64_t>(32, part_words / (6 * (int64_t)std::max(nsys, 1))));
  float *fpart = reinterpret_cast<float *>(part);
  hipLaunchKernelGGL(k_sys_bbox, dim3(nsys, shares), dim3(256), 0, st, c, P.sysoff, P.sysbox,
                     P.sc, fpart);
  if (shares > 1)
    hipLaunchKernelGGL(k_sys_bbox_fold, dim3((uint32_t)cdiv(nsys, 256)), dim3(256), 0, st, fpart,
                       shares, nsys, P.sysbox);
  hipLaunchKernelGGL(k_sys_keys, dim3(grid_for(n, 4, 8192)), dim3(256), 0, st, c, n,
                     P.sysoff, nsys, r, P.sysbox, P.keysA, P.valsA);
}

void launch_invert(const uint32_t *perm, int64_t n, uint32_t *inv, hipStream_t st) {
  hipLaunchKernelGGL(k_invert, dim3(grid_for(n, 4, 8192)), dim3(256), 0, st, perm, n, inv);
}

void launch_keys(const Coords &c, int64_t n, DevScalars *sc, uint64_t *keys, uint32_t *vals,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_keys, dim3(grid_for(n, 4, 8192)), dim3(256), 0, st, c, n, sc, keys,
                     vals);
}

void launch_gather(const Coords &c, const uint32_t *perm, int64_t n, float4 *xyzm,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_gather, dim3(grid_for(n, 4, 8192)), dim3(256), 0, st, c, perm, n,
                     xyzm);
}

}  // namespace nb
