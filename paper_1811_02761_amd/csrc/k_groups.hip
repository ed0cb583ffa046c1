// k_groups.hip -- per-group bounds for the group-wise acceleration MAC (Eq. 2).
//
// For each walked group: the members' bounding box (exact FP32 min/max),
// the smallest member |a_old| (correctly rounded sqrt of the FP32 sum of
// squares, or the key-ordered mirror's w) and delta_acc times it; gbox[2g] =
// (lo, delta_acc |a_old|min), gbox[2g + 1] = (hi, |a_old|min). Without a_old
// (bootstrap) both acceleration words are 0.
#include "nbody_internal.h"

namespace nb {

__global__ __launch_bounds__(256) void k_group_bounds(
    const DevScalars *__restrict__ sc, const uint32_t *__restrict__ queue,
    const uint32_t *__restrict__ gbegin,
    const uint32_t *__restrict__ gcount, const float4 *__restrict__ xyzm,
    const uint32_t *__restrict__ perm, const float *__restrict__ axo,
    const float *__restrict__ ayo, const float *__restrict__ azo,
    const float4 *__restrict__ asort, float delta_acc,
    float4 *__restrict__ gbox) {
  // the queued groups (block steps) or every group
  const uint32_t nq = queue ? sc->nqueue : sc->ngroup;
  const uint32_t wstride = gridDim.x * (blockDim.x >> 6);
  // wave-uniform loop (scalar index): the wave reductions below run with
  // every lane active, and the results are stored by every lane
  const uint32_t q0 = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) +
                                                     (threadIdx.x >> 6));
  for (uint32_t q = q0; q < nq; q += wstride) {
    const uint32_t g = queue ? queue[q] : q;
    const uint32_t b = gbegin[g], c = gcount[g];
    const uint32_t k = lane_id();
    const bool ok = k < c;
    const float4 p = xyzm[b + (ok ? k : 0)];
    float lx = p.x, ly = p.y, lz = p.z;
    float amin = INFINITY;
    if (asort && ok) {  // key-ordered copy of a_old with |a| in w
      amin = asort[b + k].w;
    } else if (axo && ok) {
      const uint32_t o = perm ? perm[b + k] : b + k;  // no perm: a_old in key order
      const float ax = axo[o], ay = ayo[o], az = azo[o];
      amin = sqrt_rn(__builtin_fmaf(az, az, __builtin_fmaf(ay, ay, ax * ax)));
    }
    const float hx = wave_max(lx), hy = wave_max(ly), hz = wave_max(lz);
    lx = wave_min(lx);
    ly = wave_min(ly);
    lz = wave_min(lz);
    amin = axo ? wave_min(amin) : 0.0f;
    const float dA = delta_acc * amin;
    gbox[2 * g] = make_float4(lx, ly, lz, dA);
    gbox[2 * g + 1] = make_float4(hx, hy, hz, amin);
  }
}

void launch_group_bounds(const float *axo, const float *ayo, const float *azo,
                         const float4 *asort, const uint32_t *perm, int64_t n,
                         float delta_acc, bool queued, const Ptrs &P, hipStream_t st) {
  int64_t g = cdiv(n, 4 * 8);  // up to n groups, 4 waves per block
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_group_bounds, dim3(g), dim3(256), 0, st, P.sc,
                     queued ? P.order : nullptr, P.gbegin, P.gcount, P.xyzm, perm, axo, ayo,
                     azo, asort, delta_acc, P.gbox);
}

}  // namespace nb
