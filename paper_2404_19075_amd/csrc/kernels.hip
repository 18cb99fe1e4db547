// kernels.hip -- the small kernels of one DINR training step and the launchers
// (the fused MLP kernel is in mlp.h / mlp_inst.hip, the weight gradient in
// wgrad.hip).
//
//   k_rays       per projection: index -> view/pixel -> its D x D rays, FOV clip,
//                sample counts
//   k_bundle     projection = sum of its rays' weighted sums (D > 1)
//   k_expand     upstream gradient of each ray = that of its projection (D > 1)
//   k_scan_*     exclusive scan of sample counts -> ragged point offsets
//   k_tiles      first ray of every point tile
//   k_pack       FP32 parameters -> matrix-core operand fragments (W and W^T)
//   k_fixup      ray-sums of rays that cross tile boundaries (compensated)
//   k_loss*      residuals, FP64 loss, upstream gradient 2(pbar-p)/R
//   k_reduce     compensated sum of the split partials, FP64 ||g||^2
//   k_adam       Adam update guarded by a finiteness check
#include "dinr_dev.h"
#include "kernels.h"
#include "ray_dev.h"

namespace dinr {


// One thread per projection: its D x D rays (Appendix A), ray k = b D + a to
// the centre of sub-pixel (b, a), at records r D^2 + k.  n_out[r] = |Phi_r|,
// the samples of all of them.
// pad_n > 0: every ray record is given pad_n points in the point layout
// (nray), also a ray that misses the field of view or belongs to an invalid
// index; such rays keep weight 0, so their points add nothing (the grouped
// one-pass step needs every projection to span the same number of tiles).
__global__ void k_rays(GeomDev g, const int64_t* __restrict__ idx, int64_t R,
                       RayRec* __restrict__ rays, int32_t* __restrict__ nray,
                       int32_t* __restrict__ n_out, int pad_n) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const int D = g.sub, D2 = D * D;
  const int64_t i = idx[r];
  const int64_t N = (int64_t)g.rows * g.cols;
  if (i < 0 || i >= N * g.n_views) {
    RayRec rec;
    rec.px = rec.py = rec.pz = rec.s_in = 0.f;
    rec.dx = rec.dy = rec.dz = rec.dl = 0.f;
    rec.tn = 0.f;
    rec.wgt = 0.f;
    rec.n = 0;
    rec.flags = 1;
    rec.ctr1 = rec.ctr2 = rec.ctr3 = rec.pad = 0u;
    for (int k = 0; k < D2; ++k) {
      rays[r * D2 + k] = rec;
      nray[r * D2 + k] = pad_n;
    }
    if (n_out) n_out[r] = 0;
    return;
  }
  const int m = (int)(i / N);
  const int64_t pix = i - (int64_t)m * N;
  const int row = (int)(pix / g.cols);
  const int col = (int)(pix - (int64_t)row * g.cols);
  const float u = ((float)col - 0.5f * (float)(g.cols - 1)) * g.pitch_u + g.off_u;
  const float v = ((float)row - 0.5f * (float)(g.rows - 1)) * g.pitch_v + g.off_v;
  const uint32_t i_lo = (uint32_t)((uint64_t)i & 0xFFFFFFFFu), i_hi = (uint32_t)((uint64_t)i >> 32);
  if (D == 1) {
    RayRec rec = make_ray(g, u, v, g.cth[m], g.sth[m], g.tnorm[m], g.samp_mode, g.samp_n);
    rec.ctr1 = 0u;
    rec.ctr2 = i_lo;
    rec.ctr3 = i_hi;
    rays[r] = rec;
    nray[r] = pad_n > 0 ? pad_n : rec.n;
    if (n_out) n_out[r] = rec.n;
    return;
  }
  // sub-pixel centre offsets (k % D + 1/2) / D - 1/2 in pixels
  auto sub_u = [&](int k) { return u + (float)(2 * (k % D) + 1 - D) / (float)(2 * D) * g.pitch_u; };
  auto sub_v = [&](int k) { return v + (float)(2 * (k / D) + 1 - D) / (float)(2 * D) * g.pitch_v; };
  int n_phi = 0;
  for (int k = 0; k < D2; ++k)
    n_phi += make_ray(g, sub_u(k), sub_v(k), g.cth[m], g.sth[m], g.tnorm[m], g.samp_mode,
                      g.samp_n).n;
  for (int k = 0; k < D2; ++k) {
    RayRec rec = make_ray(g, sub_u(k), sub_v(k), g.cth[m], g.sth[m], g.tnorm[m], g.samp_mode,
                          g.samp_n, n_phi);
    rec.ctr1 = (uint32_t)k;
    rec.ctr2 = i_lo;
    rec.ctr3 = i_hi;
    rays[r * D2 + k] = rec;
    nray[r * D2 + k] = pad_n > 0 ? pad_n : rec.n;
  }
  if (n_out) n_out[r] = n_phi;
}

// pbar of each projection: the sum of its D^2 rays' weighted sums (the
// weights already carry 1/|Phi|), added in FP64 and rounded once.
__global__ void k_bundle(const float* __restrict__ ray_proj, int64_t R, int D2,
                         float* __restrict__ proj) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  double acc = 0.0;
  for (int k = 0; k < D2; ++k) acc += (double)ray_proj[r * D2 + k];
  proj[r] = (float)acc;
}

// dL/d(ray sum) of each ray = dL/dpbar of its projection.
__global__ void k_expand(const float* __restrict__ g_proj, int64_t R, int D2,
                         float* __restrict__ g_ray) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= R * D2) return;
  g_ray[q] = g_proj[q / D2];
}

// Exclusive scan of n[R] into off[R+1] in three launches: every workgroup
// sums a segment of SCAN_SEG counts, one workgroup scans those sums, then
// every workgroup scans its segment from its offset.  Each thread owns
// SCAN_PER consecutive counts.
constexpr int SCAN_T = 256, SCAN_PER = 16, SCAN_SEG = SCAN_T * SCAN_PER;

__device__ inline int64_t block_incl_scan(int64_t v, int64_t* s) {
  const int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int o = 1; o < SCAN_T; o <<= 1) {
    const int64_t add = t >= o ? s[t - o] : 0;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  return s[t];
}

__global__ __launch_bounds__(SCAN_T) void k_scan_sums(const int32_t* __restrict__ n, int64_t R,
                                                       int64_t* __restrict__ bsum) {
  __shared__ int64_t s[SCAN_T];
  const int64_t i0 = (int64_t)blockIdx.x * SCAN_SEG + (int64_t)threadIdx.x * SCAN_PER;
  int64_t acc = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k)
    if (i0 + k < R) acc += n[i0 + k];
  const int64_t tot = block_incl_scan(acc, s);
  if (threadIdx.x == SCAN_T - 1) bsum[blockIdx.x] = tot;
}

// bsum[0..nb) -> exclusive prefix sums in place; *total = their sum (one
// workgroup: nb is at most 2^31 / SCAN_SEG).
__global__ __launch_bounds__(1024) void k_scan_top(int64_t* __restrict__ bsum, int64_t nb,
                                                    int64_t* __restrict__ total) {
  __shared__ int64_t s[1024];
  const int t = threadIdx.x;
  const int64_t per = (nb + 1023) / 1024;
  const int64_t b = t * per, e = (b + per < nb) ? b + per : nb;
  int64_t acc = 0;
  for (int64_t k = b; k < e; ++k) acc += bsum[k];
  s[t] = acc;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int64_t add = (t >= o) ? s[t - o] : 0;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  int64_t run = s[t] - acc;
  for (int64_t k = b; k < e; ++k) {
    const int64_t v = bsum[k];
    bsum[k] = run;
    run += v;
  }
  if (t == 1023) *total = s[1023];
}

__global__ __launch_bounds__(SCAN_T) void k_scan_apply(const int32_t* __restrict__ n, int64_t R,
                                                        const int64_t* __restrict__ bsum,
                                                        int64_t* __restrict__ off) {
  __shared__ int64_t s[SCAN_T];
  const int64_t i0 = (int64_t)blockIdx.x * SCAN_SEG + (int64_t)threadIdx.x * SCAN_PER;
  int32_t v[SCAN_PER];
  int64_t acc = 0;
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {
    v[k] = i0 + k < R ? n[i0 + k] : 0;
    acc += v[k];
  }
  int64_t run = bsum[blockIdx.x] + block_incl_scan(acc, s) - acc;
#pragma unroll
  for (int k = 0; k < SCAN_PER; ++k) {
    if (i0 + k < R) off[i0 + k] = run;
    run += v[k];
  }
}

// tile_ray0[t] = ray holding point t*TILE (R when past the last point).
__global__ void k_tiles(const int64_t* __restrict__ off, int64_t R, int tile, int64_t n_tiles_max,
                        int32_t* __restrict__ tr0) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t > n_tiles_max) return;
  const int64_t p = t * tile;
  const int64_t P = off[R];
  if (p >= P) {
    tr0[t] = (int32_t)R;
    return;
  }
  int64_t lo = 0, hi = R - 1;  // largest r with off[r] <= p
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= p) lo = mid; else hi = mid - 1;
  }
  tr0[t] = (int32_t)lo;
}

// ------------------------------------------------------------ packing
//
// Fragment of output block ob and K-chunk c for lane l, element e:
//   Wpk[((ob*CH + c)*64 + l)*VPC + e] = W[32 ob + l%32][feat(VPC c + e, l/32)]
// where CH = fan_in/(2 VPC).  The transposed copy used by the adjoint chain
// packs W_l^T the same way.
template <int PREC>
__global__ void k_pack(PackArgs a, const float* __restrict__ P, void* __restrict__ Wpk_,
                       void* __restrict__ WTpk_, float* __restrict__ bias,
                       float* __restrict__ wo_perm) {
  using T = Prec<PREC>;
  using E = typename T::elem_t;
  E* Wpk = (E*)Wpk_;
  E* WTpk = (E*)WTpk_;
  constexpr int VPC = T::VPC;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int H = a.H;
  // forward fragments
  if (gid < a.n_w) {
    int l = 0;
    while (l + 1 < a.L && gid >= a.pk_off[l + 1]) ++l;
    const int64_t q = gid - a.pk_off[l];
    const int fin = (l == 0) ? a.IN : H;
    const int CH = fin / (2 * VPC);
    const int e = (int)(q % VPC);
    const int lane = (int)((q / VPC) % 64);
    const int64_t fc = q / (VPC * 64);
    const int c = (int)(fc % CH);
    const int ob = (int)(fc / CH);
    const int row = 32 * ob + (lane & 31);
    const int k = feat(VPC * c + e, lane >> 5);
    Wpk[gid] = (E)P[a.w_off[l] + (int64_t)row * fin + k];
  }
  // transposed fragments of layers 2..L (rows = layer input units)
  if (gid < a.n_wt) {
    int l = 1;
    while (l + 1 < a.L && gid >= a.pkT_off[l + 1]) ++l;
    const int64_t q = gid - a.pkT_off[l];
    const int CH = H / (2 * VPC);
    const int e = (int)(q % VPC);
    const int lane = (int)((q / VPC) % 64);
    const int64_t fc = q / (VPC * 64);
    const int c = (int)(fc % CH);
    const int ob = (int)(fc / CH);
    const int row = 32 * ob + (lane & 31);   // input unit of layer l
    const int k = feat(VPC * c + e, lane >> 5);  // output unit of layer l
    WTpk[gid] = (E)P[a.w_off[l] + (int64_t)k * H + row];
  }
  if (gid < (int64_t)a.L * H) {
    const int l = (int)(gid / H), r = (int)(gid % H);
    bias[gid] = P[a.b_off[l] + r];
  }
  if (gid < H) {
    const int hf = (int)(gid / (H / 2)), rho = (int)(gid % (H / 2));
    wo_perm[gid] = P[a.wo_off + feat(rho, hf)];
  }
}



// Ray-sums of rays that span tiles: compensated sum of the tile partials in
// tile order.  Also writes projections of empty rays (0) and of rays with an
// out-of-range index (NaN).
__global__ void k_fixup(const RayRec* __restrict__ rays, const int64_t* __restrict__ off, int64_t R,
                        int tile, const float* __restrict__ part, float* __restrict__ proj) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const RayRec rr = rays[r];
  if (rr.flags & 1) { proj[r] = __builtin_nanf(""); return; }
  if (rr.n == 0) { proj[r] = 0.f; return; }
  const int64_t o0 = off[r], o1 = off[r + 1];
  const int64_t t0 = o0 / tile, t1 = (o1 - 1) / tile;
  if (t0 == t1) return;
  float s = part[2 * t0 + 1], comp = 0.f;
  for (int64_t k = t0 + 1; k <= t1; ++k) {
    const float y = part[2 * k] - comp;
    const float tt = s + y;
    comp = (tt - s) - y;
    s = tt;
  }
  proj[r] = __fmul_rn(rr.wgt, s);
}

// Loss (Eq. (5)) in FP64 and the upstream gradient g_r = 2 (pbar_r - p_r) / R,
// in two launches with a fixed order of summation: LOSS_BLOCKS(R) workgroups
// each sum the squared residuals of a fixed set of rays into lsum[block],
// then one workgroup adds lsum in order.
constexpr int LOSS_T = 256, LOSS_MAX_BLOCKS = LOSS_SCRATCH;
static_assert(LOSS_MAX_BLOCKS <= LOSS_T, "k_loss_total sums the partials with one thread each");
inline int loss_blocks(int64_t R) {
  const int64_t b = (R + LOSS_T - 1) / LOSS_T;
  return (int)(b < 1 ? 1 : b > LOSS_MAX_BLOCKS ? LOSS_MAX_BLOCKS : b);
}

__device__ inline void block_sum_store(double acc, double* out) {
  __shared__ double s[LOSS_T];
  const int t = threadIdx.x;
  s[t] = acc;
  __syncthreads();
  for (int o = LOSS_T / 2; o > 0; o >>= 1) {
    if (t < o) s[t] += s[t + o];
    __syncthreads();
  }
  if (t == 0) *out = s[0];
}

__global__ __launch_bounds__(LOSS_T) void k_loss(const float* __restrict__ proj,
                                                  const float* __restrict__ meas, int64_t R,
                                                  float* __restrict__ g, double* __restrict__ lsum) {
  double acc = 0.0;
  const float inv = 2.0f / (float)R;
  for (int64_t r = (int64_t)blockIdx.x * LOSS_T + threadIdx.x; r < R;
       r += (int64_t)gridDim.x * LOSS_T) {
    const float e = proj[r] - meas[r];
    acc += (double)e * (double)e;
    g[r] = inv * e;
  }
  block_sum_store(acc, lsum + blockIdx.x);
}

// Loss of the fused pass: the MLP kernel's per-workgroup sums of squared
// residuals, plus rays that hold no samples (prediction 0, so the residual
// is the measurement) and rays with an invalid index (NaN).
__global__ __launch_bounds__(LOSS_T) void k_loss_fused(const RayRec* __restrict__ rays,
                                                        const float* __restrict__ meas, int64_t R,
                                                        const double* __restrict__ lpart,
                                                        int64_t n_lpart, float* __restrict__ proj,
                                                        double* __restrict__ lsum) {
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * LOSS_T;
  const int64_t t0 = (int64_t)blockIdx.x * LOSS_T + threadIdx.x;
  for (int64_t k = t0; k < n_lpart; k += stride) acc += lpart[k];
  for (int64_t r = t0; r < R; r += stride) {
    const int32_t n = rays[r].n, flags = rays[r].flags;
    if (flags & 1) {
      proj[r] = __builtin_nanf("");
      acc += (double)__builtin_nanf("");
    } else if (n == 0) {
      proj[r] = 0.f;
      acc += (double)meas[r] * (double)meas[r];
    }
  }
  block_sum_store(acc, lsum + blockIdx.x);
}

__global__ __launch_bounds__(LOSS_T) void k_loss_total(const double* __restrict__ lsum, int nb,
                                                        int64_t R, double* __restrict__ loss) {
  __shared__ double s[LOSS_T];
  const int t = threadIdx.x;
  s[t] = t < nb ? lsum[t] : 0.0;
  __syncthreads();
  for (int o = LOSS_T / 2; o > 0; o >>= 1) {
    if (t < o) s[t] += s[t + o];
    __syncthreads();
  }
  if (t == 0) *loss = s[0] / (double)R;
}


// grad[k] = compensated sum over valid split partials (hidden layers) or over
// the per-workgroup output-layer partials; per-block FP64 sums of grad^2.
// Hidden-layer sums run over the stash chunks, one launch each, with the
// running sum and its compensation kept in a.state between launches.
__global__ __launch_bounds__(256) void k_reduce(RedArgs a) {
  __shared__ double s[256];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double sq = 0.0;
  if (k < a.np) {
    float sum = 0.f, comp = 0.f;
    if (k < a.nh) {
      if (!a.first) {
        sum = a.state[k];
        comp = a.state[a.nh + k];
      }
      const int64_t P = a.off[a.R];
      const int64_t n_tiles = (P + a.tile - 1) / a.tile;
      const int64_t pend = n_tiles * a.tile;
      const int64_t p0 = a.chunk * a.chunk_points;
      if (p0 < pend) {
        const int64_t pe = (pend < p0 + a.chunk_points) ? pend : p0 + a.chunk_points;
        const int64_t nblk = (pe - p0) / 32;
        const int64_t nsp = (nblk + a.kb - 1) / a.kb;
        // eight loads in flight, then the eight steps in split order
        const float* src = a.wpart + k;
        int64_t i = 0;
        for (; i + 8 <= nsp; i += 8) {
          float x[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) x[u] = __builtin_nontemporal_load(src + (i + u) * a.nh);
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const float y = x[u] - comp;
            const float t = sum + y;
            comp = (t - sum) - y;
            sum = t;
          }
        }
        for (; i < nsp; ++i) {
          const float y = src[i * a.nh] - comp;
          const float t = sum + y;
          comp = (t - sum) - y;
          sum = t;
        }
      }
      if (!a.last) {
        a.state[k] = sum;
        a.state[a.nh + k] = comp;
      }
    } else if (a.last) {
      const int64_t j = k - a.nh;
      for (int64_t i = 0; i < a.n_opart; ++i) {
        const float y = a.opart[i * a.no + j] - comp;
        const float t = sum + y;
        comp = (t - sum) - y;
        sum = t;
      }
    }
    if (a.last) {
      a.grad[k] = sum;
      sq = (double)sum * (double)sum;
    }
  }
  if (!a.last) return;  // uniform over the grid

  s[threadIdx.x] = sq;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.gn_part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(256) void k_gnorm(const double* __restrict__ gn_part, int64_t n,
                                               double* __restrict__ gnorm_ws,
                                               double* __restrict__ gnorm_out) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += 256) acc += gn_part[k];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *gnorm_ws = s[0];
    if (gnorm_out) *gnorm_out = s[0];
  }
}

// Adam (bias-corrected) on the flat parameters, skipped when the loss or the
// gradient norm is not finite; status[0] = 1 records the skip.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2, const double* __restrict__ loss,
                       const double* __restrict__ gnorm, int32_t* __restrict__ status) {
  const double L = *loss, G = *gnorm;
  const bool ok = isfinite(L) && isfinite(G);
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) status[0] = ok ? 0 : 1;
  if (!ok || k >= n) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.f - b1) * gk;
  const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

// ------------------------------------------------------------ launchers

#define DINR_SHAPES(X) X(128, 64) X(256, 256)

template <int PREC>
static hipError_t pack_impl(const PackArgs& a, const float* P, void* Wpk, void* WTpk, float* bias,
                            float* wo, hipStream_t st) {
  int64_t n = a.n_w;
  if (a.n_wt > n) n = a.n_wt;
  if ((int64_t)a.L * a.H > n) n = (int64_t)a.L * a.H;
  const int bs = 256;
  hipLaunchKernelGGL(k_pack<PREC>, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, st, a, P, Wpk,
                     WTpk, bias, wo);
  return hipGetLastError();
}

hipError_t launch_pack(int prec, const PackArgs& a, const float* P, void* Wpk, void* WTpk,
                       float* bias, float* wo, hipStream_t st) {
  return prec == PREC_BF16 ? pack_impl<PREC_BF16>(a, P, Wpk, WTpk, bias, wo, st)
                           : pack_impl<PREC_F32>(a, P, Wpk, WTpk, bias, wo, st);
}

int64_t scan_blocks(int64_t n_rec) { return (n_rec + SCAN_SEG - 1) / SCAN_SEG; }

hipError_t launch_rays(const GeomDev& g, const int64_t* idx, int64_t R, RayRec* rays, int32_t* nray,
                       int32_t* n_out, int64_t* off, int tile, int64_t n_tiles_max, int32_t* tr0,
                       int64_t* scan_ws, hipStream_t st, int pad_n) {
  const int bs = 256;
  const int64_t n_rec = R * g.sub * g.sub;  // ray records
  const int64_t nb = scan_blocks(n_rec);
  if (R > 0)
    hipLaunchKernelGGL(k_rays, dim3((unsigned)((R + bs - 1) / bs)), dim3(bs), 0, st, g, idx, R, rays,
                       nray, n_out, pad_n);
  if (nb > 0)
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(SCAN_T), 0, st, nray, n_rec, scan_ws);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, scan_ws, nb, off + n_rec);
  if (nb > 0)
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SCAN_T), 0, st, nray, n_rec, scan_ws,
                       off);
  hipLaunchKernelGGL(k_tiles, dim3((unsigned)((n_tiles_max + 1 + bs - 1) / bs)), dim3(bs), 0, st,
                     off, n_rec, tile, n_tiles_max, tr0);
  return hipGetLastError();
}

hipError_t launch_bundle(const float* ray_proj, int64_t R, int D2, float* proj, hipStream_t st) {
  const int bs = 256;
  if (R > 0)
    hipLaunchKernelGGL(k_bundle, dim3((unsigned)((R + bs - 1) / bs)), dim3(bs), 0, st, ray_proj, R,
                       D2, proj);
  return hipGetLastError();
}

hipError_t launch_expand(const float* g_proj, int64_t R, int D2, float* g_ray, hipStream_t st) {
  const int bs = 256;
  if (R > 0)
    hipLaunchKernelGGL(k_expand, dim3((unsigned)((R * D2 + bs - 1) / bs)), dim3(bs), 0, st, g_proj,
                       R, D2, g_ray);
  return hipGetLastError();
}

// The k_mlp instances are compiled in separate translation units
// (mlp_inst.hip, one object per precision and mode) and dispatched here.
template <int PREC, int IN, int H>
static hipError_t mlp_dispatch(int mode, int act, const MlpArgs& a, int grid, hipStream_t st) {
  switch (mode * 2 + (act ? 1 : 0)) {
    case MODE_FWD * 2 + 0: return mlp_launch<PREC, IN, H, MODE_FWD, 0>(a, grid, st);
    case MODE_FWD * 2 + 1: return mlp_launch<PREC, IN, H, MODE_FWD, 1>(a, grid, st);
    case MODE_BWD * 2 + 0: return mlp_launch<PREC, IN, H, MODE_BWD, 0>(a, grid, st);
    case MODE_BWD * 2 + 1: return mlp_launch<PREC, IN, H, MODE_BWD, 1>(a, grid, st);
    case MODE_FUSED * 2 + 0: return mlp_launch<PREC, IN, H, MODE_FUSED, 0>(a, grid, st);
    case MODE_FUSED * 2 + 1: return mlp_launch<PREC, IN, H, MODE_FUSED, 1>(a, grid, st);
    case MODE_QUERY * 2 + 0: return mlp_launch<PREC, IN, H, MODE_QUERY, 0>(a, grid, st);
    case MODE_QUERY * 2 + 1: return mlp_launch<PREC, IN, H, MODE_QUERY, 1>(a, grid, st);
    case MODE_GROUP * 2 + 1: return mlp_launch<PREC, IN, H, MODE_GROUP, 1>(a, grid, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_mlp(int prec, int in, int h, int mode, const MlpArgs& a, int grid,
                      hipStream_t st) {
#define X(I, HH)                                                                         \
  if (in == I && h == HH)                                                                \
    return prec == PREC_BF16 ? mlp_dispatch<PREC_BF16, I, HH>(mode, a.act, a, grid, st)  \
                             : mlp_dispatch<PREC_F32, I, HH>(mode, a.act, a, grid, st);
  DINR_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_query(int prec, int in, int h, const MlpArgs& a, int grid, hipStream_t st) {
  return launch_mlp(prec, in, h, MODE_QUERY, a, grid, st);
}

hipError_t launch_fixup(const RayRec* rays, const int64_t* off, int64_t R, int tile,
                        const float* part, float* proj, hipStream_t st) {
  if (R == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fixup, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, st, rays, off, R, tile,
                     part, proj);
  return hipGetLastError();
}

hipError_t launch_loss(const float* proj, const float* meas, int64_t R, float* g, double* lsum,
                       double* loss, hipStream_t st) {
  const int nb = loss_blocks(R);
  hipLaunchKernelGGL(k_loss, dim3(nb), dim3(LOSS_T), 0, st, proj, meas, R, g, lsum);
  hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(LOSS_T), 0, st, lsum, nb, R, loss);
  return hipGetLastError();
}

hipError_t launch_loss_fused(const RayRec* rays, const float* meas, int64_t R, const double* lpart,
                             int64_t n_lpart, float* proj, double* lsum, double* loss,
                             int64_t n_div, hipStream_t st) {
  const int nb = loss_blocks(R > n_lpart ? R : n_lpart);
  hipLaunchKernelGGL(k_loss_fused, dim3(nb), dim3(LOSS_T), 0, st, rays, meas, R, lpart, n_lpart,
                     proj, lsum);
  hipLaunchKernelGGL(k_loss_total, dim3(1), dim3(LOSS_T), 0, st, lsum, nb, n_div, loss);
  return hipGetLastError();
}

hipError_t launch_reduce(const RedArgs& a, double* gnorm_ws, double* gnorm_out, hipStream_t st) {
  const unsigned nblk = (unsigned)((a.np + 255) / 256);
  hipLaunchKernelGGL(k_reduce, dim3(nblk), dim3(256), 0, st, a);
  if (a.last)
    hipLaunchKernelGGL(k_gnorm, dim3(1), dim3(256), 0, st, a.gn_part, (int64_t)nblk, gnorm_ws,
                       gnorm_out);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2, const double* loss,
                       const double* gnorm, int32_t* status, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, g, m, v, n, lr,
                     b1, b2, eps, c1, c2, loss, gnorm, status);
  return hipGetLastError();
}

}  // namespace dinr