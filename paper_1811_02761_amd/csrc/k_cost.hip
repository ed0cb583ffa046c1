// k_cost.hip -- cost model of the walk's work queue: per-group features, a
// small tanh MLP (inference, backward pass, Adam) and the queue order by
// predicted cost.
//
// Features of group g (all FP32): log2 of its particle count; log2(h +
// 2^-40) with h half the diagonal of the members' box; log2 of its mass minus
// three times the previous feature (a density); log2(1 + the members' mean
// list length from their last walk). The last one is kept per particle in
// caller order and cleared at every rebuild (0 = not walked on the current
// tree): a length measured on an aged tree overstates the work on a fresh
// one. The target is log2 of the group's interactions (members x list
// entries).
//
// The order never changes the results: a group's list and its summation
// order depend on the group alone.
#include "nbody_internal.h"

namespace nb {

constexpr float kDensityFloor = 0x1p-40f;

__device__ __forceinline__ float wave_sum_f(float v) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ uint32_t wave_sum_u(uint32_t v) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// One wavefront per group (wave-uniform loop; all lanes store the result).
__global__ __launch_bounds__(256) void k_cost_features(
    const DevScalars *__restrict__ sc, const uint32_t *__restrict__ queue,
    const uint32_t *__restrict__ gbegin, const uint32_t *__restrict__ gcount,
    const float4 *__restrict__ xyzm, const uint32_t *__restrict__ perm,
    const uint32_t *__restrict__ plast, float4 *__restrict__ feat) {
  const uint32_t nq = queue ? sc->nqueue : sc->ngroup;
  const uint32_t wstride = gridDim.x * (blockDim.x >> 6);
  const uint32_t q0 = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) +
                                                     (threadIdx.x >> 6));
  for (uint32_t q = q0; q < nq; q += wstride) {
    const uint32_t g = queue ? queue[q] : q;
    const uint32_t b = gbegin[g], c = gcount[g];
    const uint32_t k = lane_id();
    const bool ok = k < c;
    const float4 p = xyzm[b + (ok ? k : 0u)];
    const uint32_t pl = ok ? plast[perm[b + k]] : 0u;
    const float ex = wave_max(p.x) - wave_min(p.x);
    const float ey = wave_max(p.y) - wave_min(p.y);
    const float ez = wave_max(p.z) - wave_min(p.z);
    const float mass = wave_sum_f(ok ? p.w : 0.0f);
    const uint32_t psum = wave_sum_u(pl);
    const float h = 0.5f * sqrtf(__builtin_fmaf(ez, ez, __builtin_fmaf(ey, ey, ex * ex)));
    const float f1 = log2f(h + kDensityFloor);
    float4 f;
    f.x = log2f((float)c);
    f.y = f1;
    f.z = log2f(mass) - 3.0f * f1;
    f.w = log2f(1.0f + (float)psum / (float)c);
    feat[g] = f;
  }
}

// After a walk: each walked group's list length to its members, and the
// training target. queue == nullptr: every group was walked.
__global__ __launch_bounds__(256) void k_cost_after(
    const DevScalars *__restrict__ sc, const uint32_t *__restrict__ queue,
    const uint32_t *__restrict__ gbegin, const uint32_t *__restrict__ gcount,
    const uint32_t *__restrict__ gent, const uint32_t *__restrict__ perm,
    uint32_t *__restrict__ plast, float *__restrict__ target) {
  const uint32_t nq = queue ? sc->nqueue : sc->ngroup;
  const uint32_t wstride = gridDim.x * (blockDim.x >> 6);
  const uint32_t q0 = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) +
                                                     (threadIdx.x >> 6));
  for (uint32_t q = q0; q < nq; q += wstride) {
    const uint32_t g = queue ? queue[q] : q;
    const uint32_t b = gbegin[g], c = gcount[g], e = gent[g];
    const uint32_t k = lane_id();
    if (k < c && e != 0xffffffffu) plast[perm[b + k]] = e;
    target[g] = log2f(fmaxf(1.0f, (float)c * (float)e));
  }
}

// ---------------------------------------------------------------- MLP
// Weight layout (row-major, output-major): mu[4] is[4] W1[H][4] b1[H]
// W2[H][H] b2[H] W3[H] b3. The inputs are standardised first, z = (f - mu)
// * is; mu and is are constants of the model (set from the training data),
// not trained. The network's output is a correction to the size-based
// estimate f.x + f.w (log2 of the group size times one plus the members' mean
// previous list length): prediction = net(z) + (f.x + f.w).
__host__ __device__ constexpr int mlp_np(int H) { return 8 + 7 * H + H * H + 1; }

// Forward, one thread per row; the weights are staged in LDS. rows_dev
// (optional) bounds the rows on the device.
template <int H>
__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ w, int64_t rows,
                                                     const uint32_t *__restrict__ rows_dev,
                                                     const float4 *__restrict__ feat,
                                                     float *__restrict__ y) {
  __shared__ float sw[mlp_np(H)];
  const int64_t nr = rows_dev ? min(rows, (int64_t)*rows_dev) : rows;
  if ((int64_t)blockIdx.x * blockDim.x >= nr) return;  // whole workgroup: no rows
  for (int i = threadIdx.x; i < mlp_np(H); i += blockDim.x) sw[i] = w[i];
  __syncthreads();
  const float *mu = sw, *is = sw + 4, *W1 = sw + 8, *b1 = W1 + 4 * H, *W2 = b1 + H,
              *b2 = W2 + H * H, *W3 = b2 + H, *b3 = W3 + H;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nr;
       r += (int64_t)gridDim.x * blockDim.x) {
    const float4 fr = feat[r];
    const float4 f = make_float4((fr.x - mu[0]) * is[0], (fr.y - mu[1]) * is[1],
                                 (fr.z - mu[2]) * is[2], (fr.w - mu[3]) * is[3]);
    float h1[H];
#pragma unroll
    for (int u = 0; u < H; ++u) {
      float s = b1[u];
      s = __builtin_fmaf(W1[4 * u + 0], f.x, s);
      s = __builtin_fmaf(W1[4 * u + 1], f.y, s);
      s = __builtin_fmaf(W1[4 * u + 2], f.z, s);
      s = __builtin_fmaf(W1[4 * u + 3], f.w, s);
      h1[u] = tanhf(s);
    }
    float out = b3[0];
#pragma unroll
    for (int u = 0; u < H; ++u) {
      float s = b2[u];
#pragma unroll
      for (int k = 0; k < H; ++k) s = __builtin_fmaf(W2[u * H + k], h1[k], s);
      out = __builtin_fmaf(W3[u], tanhf(s), out);
    }
    y[r] = out + (fr.x + fr.w);
  }
}

// Gradient of the mean squared error. Lane u < H of a wavefront owns hidden
// unit u; a wavefront takes rows gw, gw + nw, ... and accumulates its share
// of the gradient in registers in a fixed order, then writes it to
// partial[gw][0 .. np] (np = loss). k_mlp_reduce adds the shares in order,
// so the result is deterministic.
template <int H>
__global__ __launch_bounds__(256) void k_mlp_grad(const float *__restrict__ w, int64_t rows,
                                                  const float4 *__restrict__ feat,
                                                  const float *__restrict__ target,
                                                  float *__restrict__ partial) {
  __shared__ float sW2[H * H];
  const float *mu = w, *is = w + 4, *W1 = w + 8, *b1 = W1 + 4 * H, *W2 = b1 + H,
              *b2 = W2 + H * H, *W3 = b2 + H, *b3 = W3 + H;
  const float mu0 = mu[0], mu1 = mu[1], mu2 = mu[2], mu3 = mu[3];
  const float is0 = is[0], is1 = is[1], is2 = is[2], is3 = is[3];
  for (int i = threadIdx.x; i < H * H; i += blockDim.x) sW2[i] = W2[i];
  __syncthreads();
  const int u = lane_id();
  const bool on = u < H;
  const int uu = on ? u : 0;
  const float w10 = W1[4 * uu], w11 = W1[4 * uu + 1], w12 = W1[4 * uu + 2],
              w13 = W1[4 * uu + 3];
  const float bb1 = b1[uu], bb2 = b2[uu], w3 = on ? W3[uu] : 0.0f, bb3 = b3[0];
  const float inv_rows = 1.0f / (float)rows;
  float gW1[4] = {0.f, 0.f, 0.f, 0.f}, gb1 = 0.f, gW2[H], gb2 = 0.f, gW3 = 0.f, gb3 = 0.f,
        loss = 0.f;
#pragma unroll
  for (int k = 0; k < H; ++k) gW2[k] = 0.f;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  for (int64_t r = gw; r < rows; r += nw) {
    const float4 fr = feat[r];
    const float4 f = make_float4((fr.x - mu0) * is0, (fr.y - mu1) * is1, (fr.z - mu2) * is2,
                                 (fr.w - mu3) * is3);
    float s1 = bb1;
    s1 = __builtin_fmaf(w10, f.x, s1);
    s1 = __builtin_fmaf(w11, f.y, s1);
    s1 = __builtin_fmaf(w12, f.z, s1);
    s1 = __builtin_fmaf(w13, f.w, s1);
    const float h1 = on ? tanhf(s1) : 0.0f;
    float s2 = bb2;
#pragma unroll
    for (int k = 0; k < H; ++k) s2 = __builtin_fmaf(sW2[uu * H + k], __shfl(h1, k, 64), s2);
    const float h2 = on ? tanhf(s2) : 0.0f;
    const float yv = (bb3 + wave_sum_f(w3 * h2)) + (fr.x + fr.w);
    const float e = yv - target[r];
    const float dy = 2.0f * e * inv_rows;
    loss = __builtin_fmaf(e, e, loss);
    gb3 += dy;
    gW3 = __builtin_fmaf(dy, h2, gW3);
    const float d2 = on ? dy * w3 * (1.0f - h2 * h2) : 0.0f;
    gb2 += d2;
#pragma unroll
    for (int k = 0; k < H; ++k) gW2[k] = __builtin_fmaf(d2, __shfl(h1, k, 64), gW2[k]);
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < H; ++k) s = __builtin_fmaf(sW2[k * H + uu], __shfl(d2, k, 64), s);
    const float d1 = on ? s * (1.0f - h1 * h1) : 0.0f;
    gb1 += d1;
    gW1[0] = __builtin_fmaf(d1, f.x, gW1[0]);
    gW1[1] = __builtin_fmaf(d1, f.y, gW1[1]);
    gW1[2] = __builtin_fmaf(d1, f.z, gW1[2]);
    gW1[3] = __builtin_fmaf(d1, f.w, gW1[3]);
  }
  constexpr int np = mlp_np(H);
  float *out = partial + gw * (np + 1);
  if (u < 8) out[u] = 0.0f;  // the standardisation is not trained
  float *o = out + 8;
  if (on) {
    for (int j = 0; j < 4; ++j) o[4 * u + j] = gW1[j];
    o[4 * H + u] = gb1;
    for (int k = 0; k < H; ++k) o[5 * H + u * H + k] = gW2[k];
    o[5 * H + H * H + u] = gb2;
    o[6 * H + H * H + u] = gW3;
  }
  if (u == 0) {
    out[np - 1] = gb3;
    out[np] = loss * inv_rows;
  }
}

__global__ __launch_bounds__(256) void k_mlp_reduce(const float *__restrict__ partial, int nw,
                                                    int np1, float *__restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < np1; i += gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int q = 0; q < nw; ++q) s += partial[(int64_t)q * np1 + i];
    out[i] = s;
  }
}

// The model's input standardisation from training rows (one workgroup, FP64
// sums): mu = mean, is = 1 / max(standard deviation, 1e-6).
__global__ __launch_bounds__(256) void k_mlp_standardize(const float4 *__restrict__ feat,
                                                         int64_t rows, float *__restrict__ w) {
  __shared__ double s1[4][4], s2[4][4];
  double a[4] = {0, 0, 0, 0}, b[4] = {0, 0, 0, 0};
  for (int64_t r = threadIdx.x; r < rows; r += blockDim.x) {
    const float4 f = feat[r];
    const double v[4] = {f.x, f.y, f.z, f.w};
    for (int k = 0; k < 4; ++k) {
      a[k] += v[k];
      b[k] += v[k] * v[k];
    }
  }
  for (int k = 0; k < 4; ++k)
    for (int d = 32; d >= 1; d >>= 1) {
      a[k] += __shfl_xor(a[k], d, 64);
      b[k] += __shfl_xor(b[k], d, 64);
    }
  const int wv = threadIdx.x >> 6;
  if (lane_id() == 0)
    for (int k = 0; k < 4; ++k) {
      s1[wv][k] = a[k];
      s2[wv][k] = b[k];
    }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    double sa = 0, sb = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
      sa += s1[q][k];
      sb += s2[q][k];
    }
    const double mean = sa / (double)rows;
    const double var = fmax(sb / (double)rows - mean * mean, 0.0);
    w[k] = (float)mean;
    w[4 + k] = (float)(1.0 / fmax(sqrt(var), 1e-6));
  }
}

// Adam (Kingma and Ba 2015) in FP32; c1 = 1/(1 - b1^t), c2 = 1/(1 - b2^t).
__global__ __launch_bounds__(256) void k_adam(int64_t np, float *__restrict__ w,
                                              const float *__restrict__ g,
                                              float *__restrict__ m, float *__restrict__ v,
                                              float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  }
}

// Queue sort keys: one 8-bit digit, larger predicted cost first (quarter-octave
// buckets); equal digits keep group order in the stable digit sort, which
// covers the queue's entries only (the count is read on the device).
__global__ __launch_bounds__(256) void k_cost_keys(
    const DevScalars *__restrict__ sc, const uint32_t *__restrict__ queue, int mode,
    const float4 *__restrict__ feat, const float *__restrict__ pred,
    const float *__restrict__ target, int64_t n_upper, uint64_t *__restrict__ keys,
    uint32_t *__restrict__ vals) {
  const uint32_t nq = queue ? sc->nqueue : sc->ngroup;
  (void)n_upper;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nq;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t g = queue ? queue[i] : (uint32_t)i;
    const float4 f = feat[g];
    // mode 1: log2(count) + log2(1 + previous list length); mode 2: the
    // model; mode 3: the log2 interactions the last ordered walk recorded
    const float c = mode == 2 ? pred[g] : mode == 3 ? target[g] : f.x + f.w;
    const float q = fminf(fmaxf(c * 4.0f, 0.0f), 254.0f);  // NaN -> 0
    keys[i] = 254u - (uint32_t)q;
    vals[i] = g;
  }
}

__global__ void k_cost_qtotal(DevScalars *sc, int queued) {
  if (threadIdx.x == 0 && !queued) sc->nqueue = sc->ngroup;
}

namespace {
unsigned grid_for(int64_t n, int per_block, int cap) {
  int64_t g = cdiv(n, per_block);
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

template <int H>
void forward_h(const float *w, int64_t rows, const uint32_t *rows_dev, const float4 *feat,
               float *y, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_forward<H>, dim3(grid_for(rows, 256, 4096)), dim3(256), 0, st, w,
                     rows, rows_dev, feat, y);
}

template <int H>
void grad_h(const float *w, int64_t rows, const float4 *feat, const float *target,
            float *partial, float *out, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_grad<H>, dim3(kMlpWaves / 4), dim3(256), 0, st, w, rows, feat,
                     target, partial);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(grid_for(mlp_np(H) + 1, 256, 64)), dim3(256), 0, st,
                     partial, kMlpWaves, mlp_np(H) + 1, out);
}
}  // namespace

bool mlp_hidden_ok(int H) { return H == 8 || H == 16 || H == 32 || H == 64; }
int64_t mlp_nparams(int H) { return mlp_np(H); }

void launch_mlp_forward(int H, const float *w, int64_t rows, const uint32_t *rows_dev,
                        const float4 *feat, float *y, hipStream_t st) {
  switch (H) {
    case 8: forward_h<8>(w, rows, rows_dev, feat, y, st); break;
    case 16: forward_h<16>(w, rows, rows_dev, feat, y, st); break;
    case 32: forward_h<32>(w, rows, rows_dev, feat, y, st); break;
    case 64: forward_h<64>(w, rows, rows_dev, feat, y, st); break;
    default: break;
  }
}

void launch_mlp_grad(int H, const float *w, int64_t rows, const float4 *feat,
                     const float *target, float *partial, float *grad_loss, hipStream_t st) {
  switch (H) {
    case 8: grad_h<8>(w, rows, feat, target, partial, grad_loss, st); break;
    case 16: grad_h<16>(w, rows, feat, target, partial, grad_loss, st); break;
    case 32: grad_h<32>(w, rows, feat, target, partial, grad_loss, st); break;
    case 64: grad_h<64>(w, rows, feat, target, partial, grad_loss, st); break;
    default: break;
  }
}

void launch_adam(int64_t np, float *w, const float *g, float *m, float *v, int step, float lr,
                 float b1, float b2, float eps, hipStream_t st) {
  const float c1 = (float)(1.0 / (1.0 - pow((double)b1, (double)step)));
  const float c2 = (float)(1.0 / (1.0 - pow((double)b2, (double)step)));
  hipLaunchKernelGGL(k_adam, dim3(grid_for(np, 256, 64)), dim3(256), 0, st, np, w, g, m, v, lr,
                     b1, b2, eps, c1, c2);
}

void launch_mlp_standardize(const float4 *feat, int64_t rows, float *w, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_standardize, dim3(1), dim3(256), 0, st, feat, rows, w);
}

void launch_cost_features(int64_t n, bool queued, const uint32_t *perm, const Ptrs &P,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_cost_features, dim3(grid_for(n, 4 * 8, 8192)), dim3(256), 0, st, P.sc,
                     queued ? P.order : nullptr, P.gbegin, P.gcount, P.xyzm, perm, P.plast,
                     P.feat);
}

void launch_cost_after(int64_t n, bool queued, const uint32_t *perm, const Ptrs &P,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_cost_after, dim3(grid_for(n, 4 * 8, 8192)), dim3(256), 0, st, P.sc,
                     queued ? P.order : nullptr, P.gbegin, P.gcount, P.gent, perm, P.plast,
                     P.target);
}

void launch_cost_order(int64_t n, bool queued, int mode, int H, const Ptrs &P,
                       hipStream_t st) {
  if (mode == 2)
    launch_mlp_forward(H, P.mlpw, n, &P.sc->ngroup, P.feat, P.pred, st);
  hipLaunchKernelGGL(k_cost_keys, dim3(grid_for(n, 256 * 8, 8192)), dim3(256), 0, st, P.sc,
                     queued ? P.order : nullptr, mode, P.feat, P.pred, P.target, n, P.okeys,
                     P.qtmp);
  launch_digit_sort(n, queued ? &P.sc->nqueue : &P.sc->ngroup, 0, P.okeys, P.qtmp, P.okeys + n,
                    P.order, P.hist, st);
  hipLaunchKernelGGL(k_cost_qtotal, dim3(1), dim3(64), 0, st, P.sc, queued ? 1 : 0);
}

}  // namespace nb
