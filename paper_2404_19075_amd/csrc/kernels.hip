// kernels.hip -- gfx950 kernels of one DINR training step.
//
//   k_rays       per projection: index -> view/pixel -> its D x D rays, FOV clip,
//                sample counts
//   k_bundle     projection = sum of its rays' weighted sums (D > 1)
//   k_expand     upstream gradient of each ray = that of its projection (D > 1)
//   k_scan       exclusive scan of sample counts -> ragged point offsets
//   k_tiles      first ray of every point tile
//   k_pack       FP32 parameters -> matrix-core operand fragments (W and W^T)
//   k_mlp        per point tile: coordinates, Fourier features, the MLP on
//                matrix cores with activations resident in registers; then
//                either the segmented ray-sum (forward) or the adjoint chain
//                with operand stashes for the weight gradient (backward)
//   k_fixup      ray-sums of rays that cross tile boundaries (compensated)
//   k_loss       residuals, FP64 loss, upstream gradient 2(pbar-p)/R
//   k_wgrad      dW = sum_p delta_p h_p^T over the stash, split over points
//   k_reduce     compensated sum of the split partials, FP64 ||g||^2
//   k_adam       Adam update guarded by a finiteness check
#include "dinr_dev.h"
#include "kernels.h"

namespace dinr {

// ------------------------------------------------------------------ rays
//
// Ray of projection index i (Sec. II): m = i / N, n = i mod N.  The ray is
// parametrised from its point closest to the origin (for the cone beam
// p0 = d x (o x d), which has no cancellation), so sample positions stay O(1)
// in FP32.  Object rotation by theta equals rotating the source-detector pair
// by -theta about z.  Coordinates are stored already normalised to [-1,1]
// (Appendix B item 1).
// Ray through detector position (u, v) of a view rotated by theta (c = cos,
// s = sin), clipped to the FOV, with its sample count (fixed n, or
// clamp(ceil(l/h)) when samp_mode = 1).  Its weight is mu0 l / |Phi|, with
// |Phi| = n_phi, the samples of all rays of the projection (Appendix A), or
// the ray's own n when n_phi is 0.
__device__ inline RayRec make_ray(const GeomDev& g, float u, float v, float c, float s, float tn,
                                  int samp_mode, int samp_n, int n_phi = 0) {
  float p0x, p0y, p0z, d0x, d0y, d0z;
  if (g.kind == 0) {
    p0x = 0.f; p0y = u; p0z = v;
    d0x = 1.f; d0y = 0.f; d0z = 0.f;
  } else {
    const float nrm = sqrtf(g.sdd * g.sdd + u * u + v * v);
    d0x = g.sdd / nrm; d0y = u / nrm; d0z = v / nrm;
    p0x = -g.sod * (d0y * d0y + d0z * d0z);
    p0y = g.sod * d0x * d0y;
    p0z = g.sod * d0x * d0z;
  }
  const float px = c * p0x + s * p0y, py = -s * p0x + c * p0y, pz = p0z;
  const float dx = c * d0x + s * d0y, dy = -s * d0x + c * d0y, dz = d0z;
  // FOV clip
  float lo = -INFINITY, hi = INFINITY;
  bool miss = false;
  if (g.fov_kind == 0) {
    const float o[3] = {px, py, pz}, d[3] = {dx, dy, dz};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const float b0 = g.fov[2 * ax], b1 = g.fov[2 * ax + 1];
      if (d[ax] == 0.f) {
        if (o[ax] < b0 || o[ax] > b1) miss = true;
      } else {
        float ta = (b0 - o[ax]) / d[ax], tb = (b1 - o[ax]) / d[ax];
        lo = fmaxf(lo, fminf(ta, tb));
        hi = fminf(hi, fmaxf(ta, tb));
      }
    }
  } else {
    const float Rc = g.fov[0], z0 = g.fov[1], z1 = g.fov[2];
    const float qa = dx * dx + dy * dy;
    const float qb = px * dx + py * dy;  // half of the linear coefficient
    const float qc = px * px + py * py - Rc * Rc;
    if (qa == 0.f) {
      if (qc > 0.f) miss = true;
    } else {
      const float disc = qb * qb - qa * qc;
      if (disc <= 0.f) {
        miss = true;
      } else {
        const float sq = sqrtf(disc);
        lo = (-qb - sq) / qa;
        hi = (-qb + sq) / qa;
      }
    }
    if (dz == 0.f) {
      if (pz < z0 || pz > z1) miss = true;
    } else {
      float ta = (z0 - pz) / dz, tb = (z1 - pz) / dz;
      lo = fmaxf(lo, fminf(ta, tb));
      hi = fminf(hi, fmaxf(ta, tb));
    }
  }
  const float len = (!miss && hi > lo) ? hi - lo : 0.f;
  int n = 0;
  if (len > 0.f) {
    if (samp_mode == 0) {
      n = samp_n;
    } else {
      float q = ceilf(len / g.samp_h);
      q = fminf(fmaxf(q, (float)g.samp_min), (float)g.samp_max);
      n = (int)q;
    }
  }
  RayRec rec;
  rec.px = px * g.sc[0] + g.oc[0];
  rec.py = py * g.sc[1] + g.oc[1];
  rec.pz = pz * g.sc[2] + g.oc[2];
  rec.dx = dx * g.sc[0];
  rec.dy = dy * g.sc[1];
  rec.dz = dz * g.sc[2];
  rec.s_in = (n > 0) ? lo : 0.f;
  rec.dl = (n > 0) ? len / (float)n : 0.f;
  rec.tn = tn;
  rec.wgt = (n > 0) ? g.mu0 * len / (float)(n_phi > 0 ? n_phi : n) : 0.f;
  rec.n = n;
  rec.flags = 0;
  rec.ctr1 = rec.ctr2 = rec.ctr3 = rec.pad = 0u;
  return rec;
}

// One thread per projection: its D x D rays (Appendix A), ray k = b D + a to
// the centre of sub-pixel (b, a), at records r D^2 + k.  n_out[r] = |Phi_r|,
// the samples of all of them.
__global__ void k_rays(GeomDev g, const int64_t* __restrict__ idx, int64_t R,
                       RayRec* __restrict__ rays, int32_t* __restrict__ nray,
                       int32_t* __restrict__ n_out) {
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
      nray[r * D2 + k] = 0;
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
    nray[r] = rec.n;
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
    nray[r * D2 + k] = rec.n;
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

// Exclusive scan of n[R] into off[R+1] (one workgroup; R is at most a few
// million, so a single pass of per-thread serial sums is enough).
__global__ __launch_bounds__(1024) void k_scan(const int32_t* __restrict__ n, int64_t R,
                                                int64_t* __restrict__ off) {
  __shared__ int64_t s[1024];
  const int t = threadIdx.x;
  const int64_t per = (R + 1023) / 1024;
  const int64_t b = t * per, e = (b + per < R) ? b + per : R;
  int64_t acc = 0;
  for (int64_t k = b; k < e; ++k) acc += n[k];
  s[t] = acc;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    int64_t add = (t >= o) ? s[t - o] : 0;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  int64_t run = s[t] - acc;  // exclusive prefix of this thread's range
  for (int64_t k = b; k < e; ++k) {
    off[k] = run;
    run += n[k];
  }
  if (t == 1023) off[R] = s[1023];
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

// ------------------------------------------------------------ the MLP

template <int PREC>
__device__ inline void sincos_rev(float f, float* s, float* c) {
  // f in [-1/2, 1/2] revolutions
  if (PREC == PREC_BF16) {
    *s = __builtin_amdgcn_sinf(f);
    *c = __builtin_amdgcn_cosf(f);
  } else {
    sincospif(2.0f * f, s, c);
  }
}

// Phase u = b . (t, z, y, x) of one GRFF row at a normalised point, reduced
// to [-1/2, 1/2] revolutions (App. B item 2).  The forward and the layer-1
// weight gradient both evaluate the encoding through this function, so the
// gradient sees the very values the forward used.
__device__ inline float grff_phase(float4 b, float rt, float rz, float ry, float rx) {
  const float u = b.x * rt + b.y * rz + b.z * ry + b.w * rx;
  return u - rintf(u);
}

// ---- weight panels in LDS
//
// Every layer's packed fragments are streamed through two LDS buffers of
// PANEL_BYTES in "panels" of OBP output blocks: while the wave computes one
// panel, the workgroup's global->LDS DMA (buffer loads with the LDS bit) fills the
// other with the next panel of the sequence (the next layer's first panel at
// the end of a layer, the first layer of the next tile at the end of a tile).
// One barrier per panel: after it, the panel just waited for is visible to
// all waves and the other buffer is no longer being read.
constexpr int PANEL_BYTES = 32768;

// Output blocks per panel: as many as fit, but at most half the layer, so that
// every layer has an even number of panels and starts in buffer 0.  The buffer
// a panel lives in is then known at compile time, and the two buffers being
// distinct LDS objects lets the compiler see that reading one does not have to
// wait for the DMA into the other.
template <int KC, int H>
__host__ __device__ constexpr int panel_obs() {
  return (PANEL_BYTES / (KC * 1024)) > H / 64 ? H / 64
         : (PANEL_BYTES / (KC * 1024)) < 1     ? 1
                                                : PANEL_BYTES / (KC * 1024);
}
template <int KC, int H>
__host__ __device__ constexpr int panel_bytes() { return panel_obs<KC, H>() * KC * 1024; }

typedef __attribute__((address_space(3))) void lds_void;

// A per-lane byte offset the optimizer cannot see through: it is recomputed
// where it is used (one VALU op from the lane id) instead of being hoisted
// out of the tile loop as one 64-bit address per panel, which would not fit
// in registers and would come back from scratch memory.
__device__ inline uint32_t lane_off(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Forces a 16-byte chunk to be computed at this point of the program (an
// opaque use ordered with the other volatile asm, e.g. the panel barrier).
template <class C>
__device__ inline void pin(C& v) {
  static_assert(sizeof(C) == 16, "16-byte chunk");
  typedef int i32x4 __attribute__((ext_vector_type(4)));
  i32x4 t = __builtin_bit_cast(i32x4, v);
  asm volatile("" : "+v"(t));
  v = __builtin_bit_cast(C, t);
}

// A position in a DMA source: a buffer resource over one device array and a
// byte offset into it (off < 0: nothing).  The copies into LDS are MUBUF
// loads with the LDS bit: they count only on vmcnt, so the compiler keeps
// counted waits on LDS reads while they are in flight (a FLAT-encoded copy
// would make it drain the LDS queue at every read), and the hardware range
// check turns a read past the array into zeros instead of a fault.
struct WSrc {
  __amdgpu_buffer_rsrc_t r;
  int off;
  __device__ WSrc at(int delta) const { return WSrc{r, off + delta}; }
};

__device__ inline __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, int64_t bytes) {
  // raw (stride 0) buffer; word 3 selects 32-bit data for untyped loads
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}

// bytes: a multiple of 1 KB.  Wave w of nw copies the 1 KB blocks w, w+nw,
// ...; the LDS destination of one instruction is wave-uniform.
template <int NW>
__device__ inline void dma_panel(WSrc src, char* dst, int bytes, int w, int lane) {
  uint32_t lo = lane_off((uint32_t)(w * 1024 + lane * 16));
  for (int off = w * 1024; off < bytes; off += NW * 1024, lo += NW * 1024)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(src.r, (lds_void*)(dst + off), 16, (int)lo, src.off,
                                             0, 0);
}

// One layer's H biases (fp32) into LDS with a single wave instruction.
template <int H>
__device__ inline void dma_bias(WSrc src, float* dst, int lane) {
  constexpr int SZ = H * 4 / WAVE;  // bytes per lane
  static_assert(SZ == 4 || SZ == 16, "one DMA instruction per layer's biases");
  const int lo = (int)lane_off((uint32_t)(lane * SZ));
  if constexpr (SZ == 16)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(src.r, (lds_void*)dst, 16, lo, src.off, 0, 0);
  else
    __builtin_amdgcn_raw_ptr_buffer_load_lds(src.r, (lds_void*)dst, 4, lo, src.off, 0, 0);
}


// Workgroup barrier for the panel exchange.  It orders LDS traffic (and the
// DMA into LDS that each wave has already waited for) but, unlike
// __syncthreads, whose release fence waits for every outstanding global
// store, leaves the wave's stash stores in flight.
__device__ inline void panel_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Wait until at most N vector-memory operations are outstanding.  Vector
// memory operations complete in issue order, so when exactly N stash stores
// were issued after a panel's DMA, vmcnt(N) waits for that DMA but not for
// the stores: they drain while the next panel computes.
// Issued through the builtin, not inline asm, so that the compiler's own
// wait insertion knows what has completed (gfx9 encoding: vmcnt in bits 3:0
// and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at their maxima).
template <int N>
__device__ inline void wait_vm() {
  static_assert(N >= 0 && N <= 63, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Layer epilogues:
//   EPI_RELU:      y = relu(W x + b)
//   EPI_RELU_MASK: the same, and the ReLU mask bits go to msk
//   EPI_MASK:      y = (W x) . mask, the mask bits coming from msk
//   EPI_SWISH:     y = swish(W x + b) = z sigmoid(z)
//   EPI_SWISH_D:   the same, and swish'(z) goes to the derivative stash
//   EPI_DERIV:     y = (W x) . swish'(z), the derivatives read back from it
enum { EPI_RELU = 0, EPI_RELU_MASK = 1, EPI_MASK = 2, EPI_SWISH = 3, EPI_SWISH_D = 4,
       EPI_DERIV = 5 };
__host__ __device__ constexpr bool epi_forward(int e) { return e != EPI_MASK && e != EPI_DERIV; }
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Packed 16-bit integer max/min/multiply as single instructions (written out:
// the compiler otherwise turns min(max(h, 0), 1) into per-half compares and
// selects through lane masks, and splits the bf16 conversions feeding a
// 16-bit multiply into one conversion per value).
__device__ inline uint32_t pk_max0_i16(uint32_t x) {
  uint32_t r;
  asm("v_pk_max_i16 %0, %1, 0" : "=v"(r) : "v"(x));
  return r;
}
__device__ inline uint32_t pk_mul_u16(uint32_t x, uint32_t y) {
  uint32_t r;
  asm("v_pk_mul_lo_u16 %0, %1, %2" : "=v"(r) : "v"(x), "v"(y));
  return r;
}
__device__ inline uint32_t pk_min1_u16(uint32_t x) {
  uint32_t r;
  asm("v_pk_min_u16 %0, %1, %2" : "=v"(r) : "v"(x), "v"(0x00010001u));
  return r;
}

template <int PREC, int H>
__host__ __device__ constexpr int mask_words() { return Prec<PREC>::NB * (H / 32) / 2; }

// Epilogue of one 16-byte chunk of an output block: ReLU (recording mask
// bits) or the stored mask applied, then conversion to the operand type.
// 0 - x as an opaque VALU op: keeps "(-r) >> 31" a subtract and a shift
// instead of being rewritten into a compare into a lane mask and a select.
__device__ inline uint32_t neg_u32(uint32_t x) {
  uint32_t r;
  asm("v_sub_u32 %0, 0, %1" : "=v"(r) : "v"(x));
  return r;
}

template <int PREC, int H, int EPI>
__device__ inline void epi_chunk(const f32x16 (&acc)[Prec<PREC>::NB], int ob, int k,
                                 typename Prec<PREC>::chunk_t (&y)[Prec<PREC>::NB][chunks<PREC>(H)],
                                 uint32_t (&msk)[mask_words<PREC, H>()],
                                 typename Prec<PREC>::chunk_t* __restrict__ actp,
                                 const typename Prec<PREC>::chunk_t* actv, int lane) {
  using T = Prec<PREC>;
  constexpr int VPC = T::VPC, CPO = 16 / VPC, OB = H / 32;
  const int nb = k / CPO, kk = k % CPO;
  const int g = nb * OB + ob;
  const int mw = g >> 1;
  if constexpr (EPI == EPI_SWISH || EPI == EPI_SWISH_D) {
    // swish(z) = z s and swish'(z) = s (1 + z (1 - s)), s = sigmoid(z)
    // (App. B item 3); derivatives of the outputs go to the stash, rounded
    // like the operands
    float v[VPC], dv[VPC];
#pragma unroll
    for (int e = 0; e < VPC; ++e) {
      const float zz = acc[nb][kk * VPC + e];
      // v_rcp_f32 (1 ulp): a correctly rounded reciprocal is an IEEE
      // division sequence five times as long
      const float sg = __builtin_amdgcn_rcpf(1.0f + __expf(-zz));
      v[e] = zz * sg;
      dv[e] = __builtin_fmaf(v[e], 1.0f - sg, sg);  // s + z s (1 - s)
    }
    y[nb][ob * CPO + kk] = T::from_f32(v);
    if (EPI == EPI_SWISH_D)
      T::store_nt(&actp[(nb * chunks<PREC>(H) + ob * CPO + kk) * 64 + lane], T::from_f32(dv));
    return;
  } else if constexpr (EPI == EPI_DERIV) {
    float v[VPC];
#pragma unroll
    for (int e = 0; e < VPC; ++e) v[e] = acc[nb][kk * VPC + e] * T::get(actv[k], e);
    y[nb][ob * CPO + kk] = T::from_f32(v);
    return;
  }
  if constexpr (PREC == PREC_BF16) {
    // Round first, then work on the bf16 pairs, two values per register:
    // ReLU is max_i16 of the bit patterns (negative values are negative
    // integers), a unit's mask bit is min_u16(h, 1), and masking multiplies
    // each half by its 0/1 bit.  Chunk j = 2 (g & 1) + kk of a mask word keeps
    // the bits of its 4 low halves at 4j..4j+3 and of its high halves at
    // 16+4j..16+4j+3.
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = acc[nb][kk * 8 + e];
    u32x4 q = __builtin_bit_cast(u32x4, T::from_f32(v));
    const int j = 2 * (g & 1) + kk;
    if (EPI != EPI_MASK) {
      uint32_t bits = 0;
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        q[d] = pk_max0_i16(q[d]);
        if (EPI == EPI_RELU_MASK) bits |= pk_min1_u16(q[d]) << d;
      }
      if (EPI == EPI_RELU_MASK) {
        msk[mw] |= bits << (4 * j);
        // fold the bits in now: left to itself the compiler defers this to
        // the store of the mask words after the layer and keeps every
        // intermediate of the layer alive until then
        asm volatile("" : "+v"(msk[mw]));
      }
    } else {
      const uint32_t bits = msk[mw] >> (4 * j);
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        q[d] = pk_mul_u16(q[d], (bits >> d) & 0x00010001u);
      }
    }
    y[nb][ob * CPO + kk] = __builtin_bit_cast(typename T::chunk_t, q);
  } else {
    // FP32: integer VALU on the bit patterns (no compares into lane masks).
    // ReLU is max_i32(bits, 0); its mask bit (bit kk*4+e of the ob's 16) is
    // the sign of -relu (1 iff z > 0); masking ANDs the value with the
    // sign-extended bit.
    const int sh = 16 * (g & 1) + kk * VPC;
    float v[VPC];
    if (EPI != EPI_MASK) {
      uint32_t bits = 0;
#pragma unroll
      for (int e = 0; e < VPC; ++e) {
        const int zi = __float_as_int(acc[nb][kk * VPC + e]);
        const int r = zi > 0 ? zi : 0;  // v_max_i32
        v[e] = __int_as_float(r);
        if (EPI == EPI_RELU_MASK) bits |= (neg_u32((uint32_t)r) >> 31) << e;
      }
      if (EPI == EPI_RELU_MASK) {
        msk[mw] |= bits << sh;
        asm volatile("" : "+v"(msk[mw]));
      }
    } else {
      const uint32_t bits = msk[mw] >> sh;
#pragma unroll
      for (int e = 0; e < VPC; ++e) {
        const int keep = -(int)((bits >> e) & 1u);  // 0 or all ones
        v[e] = __int_as_float(__float_as_int(acc[nb][kk * VPC + e]) & keep);
      }
    }
    y[nb][ob * CPO + kk] = T::from_f32(v);
  }
}

// One fully connected layer for the wave's NB point blocks, with one of the
// epilogues above.
// W: the layer's packed fragments in global memory, streamed through LDS.
// Wnext/next_bytes: first panel of whatever follows in the sequence (or none).
// sbias: this layer's biases in LDS (EPI_RELU, EPI_RELU_MASK).  gbias_next (or
// none): biases of the next forward layer, copied into sbias_next.
// stash (nullable): where to store x for the weight gradient.
// Instruction stream per K-step: 2 MFMAs (one per point block), one LDS read
// of the fragment D steps ahead, and a slice of the previous output block's
// epilogue, so VALU work and LDS latency overlap the matrix cores.
template <int PREC, int KC, int H, int EPI, int VM_ENTRY>
__device__ inline void layer(const typename Prec<PREC>::chunk_t (&x)[Prec<PREC>::NB][KC],
                             typename Prec<PREC>::chunk_t (&y)[Prec<PREC>::NB][chunks<PREC>(H)],
                             WSrc W, WSrc Wnext, int next_bytes, const float* sbias,
                             WSrc gbias_next, float* sbias_next,
                             uint32_t (&msk)[mask_words<PREC, H>()],
                             typename Prec<PREC>::chunk_t* __restrict__ stash, char* sW0, char* sW1,
                             int lane, int w, int z,
                             typename Prec<PREC>::chunk_t* __restrict__ actp = nullptr) {
  using T = Prec<PREC>;
  using chunk_t = typename T::chunk_t;
  constexpr int NB = T::NB, VPC = T::VPC;
  constexpr int OB = H / 32;
  constexpr int CPO = 16 / VPC;  // chunks per output block and point block
  constexpr int NEPI = NB * CPO;  // epilogue chunks per output block
  constexpr int OBP = panel_obs<KC, H>();
  constexpr int PB = panel_bytes<KC, H>();
  constexpr int D = 3;  // LDS prefetch distance (K-steps)
  constexpr int MFMA_PER_STEP = (PREC == PREC_BF16 ? 1 : 4) * NB;
  constexpr int NP = OB / OBP;          // panels in this layer
  constexpr int SPP = KC / NP;          // stash chunks per point block stored per panel
  static_assert(OB % OBP == 0, "panels must tile the output blocks");
  static_assert(KC % NP == 0, "stash stores must spread evenly over the panels");
  static_assert(NP % 2 == 0, "each layer starts and ends in buffer 0");
  const int hf = lane >> 5;
  if (EPI == EPI_RELU_MASK)
#pragma unroll
    for (int k = 0; k < mask_words<PREC, H>(); ++k) msk[k] = 0u;
  f32x16 accp[NB];
  // EPI_DERIV: derivative chunk k of an output block, loaded at the K-step
  // where chunk k of the block before is consumed (one block of latency)
  chunk_t actk[NEPI];
  const char* ap = (const char*)actp + lane_off((uint32_t)(lane * sizeof(chunk_t)));
#pragma unroll
  for (int ob = 0; ob < OB; ++ob) {
    if (ob % OBP == 0) {
      const int pi = ob / OBP;
      // the panel DMA'd last is complete; stores issued after it may still drain
      // (a layer without a stash simply waits for everything outstanding)
      if (stash) {
        if (pi == 0) wait_vm<VM_ENTRY>();
        else wait_vm<NB * SPP>();
      } else {
        wait_vm<0>();
      }
      panel_barrier();
      char* nxt = (pi & 1) ? sW0 : sW1;
      // the next layer's biases: the previous reader of their buffer (two
      // layers back) finished before this layer's first barrier
      if (pi == 0 && gbias_next.off >= 0 && w == 0) dma_bias<H>(gbias_next, sbias_next, lane);
      if (ob + OBP < OB) dma_panel<T::WAVES>(W.at((pi + 1) * PB), nxt, PB, w, lane);
      else if (Wnext.off >= 0) dma_panel<T::WAVES>(Wnext, nxt, next_bytes, w, lane);
      asm volatile("" ::: "memory");  // the stores below stay after the DMA
      if (stash) {
        // this panel's share of the layer input for the weight gradient
        char* sp = (char*)stash + lane_off((uint32_t)(lane * sizeof(chunk_t)));
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int c = pi * SPP; c < (pi + 1) * SPP; ++c)
            T::store_nt((chunk_t*)(sp + (nb * KC + c) * 64 * sizeof(chunk_t)), x[nb][c]);
      }
    }
    const chunk_t* __restrict__ Wp =
        (const chunk_t*)(((ob / OBP) & 1) ? sW1 : sW0) + (ob % OBP) * KC * 64;
    f32x16 acc[NB];
    if (epi_forward(EPI)) {
      float bq[16];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 b4 = *(const float4*)(sbias + z + 32 * ob + 8 * q + 4 * hf);
        bq[4 * q + 0] = b4.x; bq[4 * q + 1] = b4.y; bq[4 * q + 2] = b4.z; bq[4 * q + 3] = b4.w;
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[nb][r] = bq[r];
    } else {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[nb][r] = 0.f;
    }
    chunk_t a[D + 1];
#pragma unroll
    for (int c = 0; c < D && c < KC; ++c) a[c] = Wp[c * 64 + lane];
    // the bias reads (forward kinds) and the first D fragment reads lead the block
    __builtin_amdgcn_sched_group_barrier(0x100, (D < KC ? D : KC) + (epi_forward(EPI) ? 4 : 0),
                                         0);
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      if (c + D < KC) a[(c + D) % (D + 1)] = Wp[(c + D) * 64 + lane];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) T::mma(acc[nb], a[c % (D + 1)], x[nb][c]);
      __builtin_amdgcn_sched_group_barrier(0x008, MFMA_PER_STEP, 0);
      if (c + D < KC) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      if (ob > 0) {
        // epilogue chunks of block ob-1 assigned to this step
#pragma unroll
        for (int k = 0; k < NEPI; ++k)
          if ((k * KC) / NEPI == c)
            epi_chunk<PREC, H, EPI>(accp, ob - 1, k, y, msk, actp, actk, lane);
      }
      if (EPI == EPI_DERIV) {
#pragma unroll
        for (int k = 0; k < NEPI; ++k)
          if ((k * KC) / NEPI == c)
            actk[k] = *(const chunk_t*)(ap + ((k / CPO) * chunks<PREC>(H) + ob * CPO + k % CPO) *
                                                 64 * sizeof(chunk_t));
      }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) accp[nb] = acc[nb];
  }
#pragma unroll
  for (int k = 0; k < NEPI; ++k) epi_chunk<PREC, H, EPI>(accp, OB - 1, k, y, msk, actp, actk, lane);
}

// ACT: 0 ReLU hidden layers (their masks stay in LDS), 1 Swish (swish'(z) of
// every layer goes through the stash in the adjoint modes)
template <int PREC, int IN, int H, int MODE, int ACT>
__global__ __launch_bounds__(Prec<PREC>::WAVES * 64, 1) void k_mlp(MlpArgs a) {
  using T = Prec<PREC>;
  using chunk_t = typename T::chunk_t;
  constexpr int NB = T::NB, VPC = T::VPC;
  constexpr int CI = chunks<PREC>(IN), CHh = chunks<PREC>(H);
  constexpr int WAVES_PER_WG = T::WAVES;
  constexpr int TILE = WAVES_PER_WG * NB * 32;
  constexpr int C = IN / 2;
  constexpr int MSK_PER_LAYER = mask_words<PREC, H>();  // 32-bit mask words per lane per layer
  constexpr int MSK_LAYERS = (MODE != MODE_FWD && ACT == 0) ? MAX_LAYERS - 1 : 1;
  constexpr int PB_IN = panel_bytes<CI, H>(), PB_H = panel_bytes<CHh, H>();
  // the wave index in a scalar register: every address derived from it
  // (stash blocks, LDS slices, DMA destinations) is then wave-uniform too
  const int lane = threadIdx.x & 63, hf = lane >> 5, pl = lane & 31;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  // weight panels: two separate arrays (see panel_obs)
  __shared__ __align__(16) char sW0[PANEL_BYTES];
  __shared__ __align__(16) char sW1[PANEL_BYTES];
  __shared__ float4 sB[C];
  __shared__ float sval[TILE];
  __shared__ int32_t srid[TILE];
  __shared__ float sg[TILE];  // fused mode: upstream gradient of the tile's rays
  __shared__ float swgt[TILE];  // query mode: weight mu0 l / n of each point's ray
  __shared__ double sloss[WAVES_PER_WG * 64];
  __shared__ float sdwo[WAVES_PER_WG][H + 1];
  // biases: layer 0 (loaded once), odd and even hidden layers (each copied in
  // during the layer before); w_o in register-slot order.  Separate arrays,
  // selected at compile time, so reads never wait for an unrelated DMA.
  __shared__ __align__(16) float sBias0[H];
  __shared__ __align__(16) float sBiasOdd[H];
  __shared__ __align__(16) float sBiasEven[H];
  __shared__ __align__(16) float sWo[H];
  // ReLU masks of h_1 .. h_{L-1} for the adjoint chain
  __shared__ uint32_t smsk[WAVES_PER_WG][MSK_LAYERS][MSK_PER_LAYER][64];

  constexpr bool QUERY = MODE == MODE_QUERY;
  const int64_t P = QUERY ? 0 : a.off[a.R];
  const int64_t n_tiles = QUERY ? a.n_qtiles : (P + TILE - 1) / TILE;
  const int64_t t_end = QUERY ? n_tiles : (a.tile_end < n_tiles ? a.tile_end : n_tiles);
  const float bo = a.params[a.bo_off];
  const int L = a.L;
  constexpr bool FWD_PART = MODE == MODE_FWD || MODE == MODE_FUSED || MODE == MODE_QUERY;
  constexpr bool BWD_PART = MODE == MODE_BWD || MODE == MODE_FUSED;
  // the adjoint needs the ReLU masks (or the Swish derivatives) of the
  // forward layers
  constexpr int FWD_EPI = ACT == 1 ? (BWD_PART ? EPI_SWISH_D : EPI_SWISH)
                                   : (BWD_PART ? EPI_RELU_MASK : EPI_RELU);
  constexpr int ADJ_EPI = ACT == 1 ? EPI_DERIV : EPI_MASK;
  double lossacc = 0.0;
  const float g_scale = 2.0f / (float)a.R;
  const __amdgpu_buffer_rsrc_t rW = buffer_rsrc(a.Wpk, a.wpk_bytes);
  const __amdgpu_buffer_rsrc_t rWT = buffer_rsrc(a.WTpk, a.wtpk_bytes);
  const __amdgpu_buffer_rsrc_t rB = buffer_rsrc(a.bias, (int64_t)L * H * sizeof(float));
  constexpr int ES = sizeof(typename T::elem_t);
  auto Wl = [&](int l) { return WSrc{rW, (int)(a.wpk_off[l] * ES)}; };
  auto WTl = [&](int l) { return WSrc{rWT, (int)(a.wtpk_off[l] * ES)}; };
  const WSrc none{rW, -1};

  const int64_t t0 = (QUERY ? 0 : a.tile_begin) + blockIdx.x;
  if (t0 < t_end) dma_panel<WAVES_PER_WG>(Wl(0), sW0, PB_IN, w, lane);
  for (int k = threadIdx.x; k < C; k += blockDim.x) sB[k] = a.Bmat[k];
  for (int k = threadIdx.x; k < H; k += blockDim.x) {
    sBias0[k] = a.bias[k];
    sWo[k] = a.wo_perm[k];
  }
  if (MODE != MODE_FWD)
    for (int k = threadIdx.x; k < WAVES_PER_WG * (H + 1); k += blockDim.x) (&sdwo[0][0])[k] = 0.f;
  __syncthreads();

  for (int64_t t = t0; t < t_end; t += gridDim.x) {
    const bool more = t + gridDim.x < t_end;
    // a zero the compiler cannot see through: keeps the per-lane loads of B
    // rows, biases and w_o inside the tile loop instead of hoisting (and
    // spilling) hundreds of loop-invariant values
    int z = 0;
    asm volatile("" : "+v"(z));
    int rid[NB];
    int poff[NB];  // first point of the point's ray, relative to the tile
    float wgt[NB];
    chunk_t x0[NB][CI];
    // ---- coordinates and Fourier features (Appendix A, Appendix B items 1-2)
    const int64_t blk0 = (t - a.tile_begin) * (TILE / 32) + w * NB;  // stash block of nb = 0
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int64_t p = t * TILE + w * (NB * 32) + nb * 32 + pl;
      float rt = 0.f, rz = 0.f, ry = 0.f, rx = 0.f;
      rid[nb] = -1;
      poff[nb] = 0;
      wgt[nb] = 0.f;
      if (QUERY) {
        const QueryTile qt = a.qtiles[t];
        const QueryDesc q = a.qdesc[qt.slot];
        const int tp = w * (NB * 32) + nb * 32 + pl;
        rt = q.tn;
        if (q.kind == 0) {
          const int64_t pq = (int64_t)qt.tile * TILE + tp;
          if (pq < (int64_t)q.n * q.n) {
            const int i = (int)(pq / q.n), j = (int)(pq - (int64_t)i * q.n);
            rz = q.zn;
            ry = -1.f + (2.f * i + 1.f) / (float)q.n;
            rx = -1.f + (2.f * j + 1.f) / (float)q.n;
            rid[nb] = (int)pq;
          }
        } else {
          const int S = q.samples;
          const int64_t ray = (int64_t)qt.tile * (TILE / S) + tp / S;
          const int j = tp % S;
          if (ray < (int64_t)q.n * q.n) {
            const int row = (int)(ray / q.n), col = (int)(ray - (int64_t)row * q.n);
            const GeomDev& g = a.geom;
            const float pu = g.pitch_u * (float)g.cols / (float)q.n;
            const float pv = g.pitch_v * (float)g.rows / (float)q.n;
            const float u = ((float)col - 0.5f * (float)(q.n - 1)) * pu + g.off_u;
            const float v = ((float)row - 0.5f * (float)(q.n - 1)) * pv + g.off_v;
            const RayRec rr = make_ray(g, u, v, q.cth, q.sth, q.tn, 0, S);
            if (rr.n > 0) {
              const float s = rr.s_in + ((float)j + 0.5f) * rr.dl;
              rz = rr.pz + s * rr.dz;
              ry = rr.py + s * rr.dy;
              rx = rr.px + s * rr.dx;
              rid[nb] = (int)(tp / S);
              wgt[nb] = rr.wgt;
            } else if (j == 0 && hf == 0) {
              q.out[ray] = 0.f;  // the ray misses the field of view
            }
          }
        }
      } else if (p < P) {
        int64_t lo = a.tile_ray0[t], hi = a.tile_ray0[t + 1];
        if (hi > a.R - 1) hi = a.R - 1;
        while (lo < hi) {
          const int64_t mid = (lo + hi + 1) >> 1;
          if (a.off[mid] <= p) lo = mid; else hi = mid - 1;
        }
        const RayRec rr = a.rays[lo];
        const int j = (int)(p - a.off[lo]);
        // midpoint, or a uniform offset in [0, 1) drawn for (j, ray, projection)
        float u = 0.5f;
        if (a.jitter)
          u = (float)(philox_word0((uint32_t)j, rr.ctr1, rr.ctr2, rr.ctr3, a.key0, a.key1) >> 8) *
              (1.0f / 16777216.0f);
        const float s = rr.s_in + ((float)j + u) * rr.dl;
        rt = rr.tn;
        rz = rr.pz + s * rr.dz;
        ry = rr.py + s * rr.dy;
        rx = rr.px + s * rr.dx;
        rid[nb] = (int)lo;
        poff[nb] = (int)(a.off[lo] - t * TILE);
        wgt[nb] = rr.wgt;
      }
      if (BWD_PART && hf == 0) {
        // the layer-1 weight gradient re-derives this point's encoding from
        // its coordinates (16 bytes instead of 2C features); padding points
        // store zeros, which encode to finite values
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 r4 = {rt, rz, ry, rx};
        __builtin_nontemporal_store(r4, (f4*)a.stash + a.h_base[0] + (blk0 + nb) * 32 + pl);
      }
#pragma unroll
      for (int c = 0; c < CI / 2; ++c) {
        float cv[VPC], sv[VPC];
#pragma unroll
        for (int e = 0; e < VPC; ++e) {
          const float f = grff_phase(sB[z + feat(VPC * c + e, hf)], rt, rz, ry, rx);
          sincos_rev<PREC>(f, &sv[e], &cv[e]);
        }
        x0[nb][c] = T::from_f32(cv);
        x0[nb][c + CI / 2] = T::from_f32(sv);
        // materialise the encoded chunk here: otherwise the arithmetic sinks
        // past the first panel barrier to its use, and the B rows of every
        // chunk stay live across it
        pin(x0[nb][c]);
        pin(x0[nb][c + CI / 2]);
      }
    }
    uint32_t* msk_w = &smsk[w][0][0][0];
    // Swish derivatives of layer l's outputs, in the layout of the stash
    auto astash = [&](int l) -> chunk_t* {
      return (BWD_PART && ACT == 1) ? (chunk_t*)a.stash + a.a_base[l] + blk0 * (CHh * 64)
                                    : nullptr;
    };
    auto hstash = [&](int l, int ch) -> chunk_t* {
      return BWD_PART ? (chunk_t*)a.stash + a.h_base[l] + blk0 * (ch * 64) : nullptr;
    };
    // what follows the last forward layer in the panel sequence
    const WSrc after_fwd = (BWD_PART && L > 1) ? WTl(L - 1) : (more ? Wl(0) : none);
    // biases of layer l+1 (none after the last layer: layer 0's stay resident)
    auto bias_next = [&](int l) -> WSrc {
      return l + 1 < L ? WSrc{rB, (l + 1) * H * (int)sizeof(float)} : none;
    };
    const int after_fwd_bytes = (BWD_PART && L > 1) ? PB_H : PB_IN;
    // ---- hidden layers (Appendix B item 3)
    chunk_t y[NB][CHh];
    {
      uint32_t mk[MSK_PER_LAYER];
      const WSrc nx = L > 1 ? Wl(1) : after_fwd;
      const int nxb = L > 1 ? PB_H : after_fwd_bytes;
      layer<PREC, CI, H, FWD_EPI, 0>(x0, y, Wl(0), nx, nxb, sBias0, bias_next(0), sBiasOdd,
                                           mk, nullptr, sW0, sW1, lane, w, z, astash(0));
      if (BWD_PART && ACT == 0 && L > 1)
#pragma unroll
        for (int k = 0; k < MSK_PER_LAYER; ++k) msk_w[(0 * MSK_PER_LAYER + k) * 64 + lane] = mk[k];
    }
    // hidden layers 2..L, two per iteration with the roles of y and z swapped
    // so that no activation array is copied between layers
    // sb: this layer's biases, sbn: where the next layer's go
    auto hidden = [&](int l, const chunk_t (&in)[NB][CHh], chunk_t (&out)[NB][CHh],
                      const float* sb, float* sbn) {
      uint32_t mk[MSK_PER_LAYER];
      const WSrc nx = (l + 1 < L) ? Wl(l + 1) : after_fwd;
      const int nxb = (l + 1 < L) ? PB_H : after_fwd_bytes;
      // stores the previous layer issued after its last DMA: its last panel's
      // share (layer 0 stores none: its input is re-derived from coordinates)
      constexpr int VM_1 = 0;
      constexpr int VM_H = BWD_PART ? NB * (CHh / (H / 32 / panel_obs<CHh, H>())) : 0;
      if (VM_1 != VM_H && l == 1)
        layer<PREC, CHh, H, FWD_EPI, VM_1>(in, out, Wl(l), nx, nxb, sb, bias_next(l), sbn, mk,
                                                 hstash(l, CHh), sW0, sW1, lane, w, z, astash(l));
      else
        layer<PREC, CHh, H, FWD_EPI, VM_H>(in, out, Wl(l), nx, nxb, sb, bias_next(l), sbn, mk,
                                                 hstash(l, CHh), sW0, sW1, lane, w, z, astash(l));
      if (BWD_PART && ACT == 0 && l < L - 1)
#pragma unroll
        for (int k = 0; k < MSK_PER_LAYER; ++k) msk_w[(l * MSK_PER_LAYER + k) * 64 + lane] = mk[k];
    };
    for (int l = 1; l < L; l += 2) {
      chunk_t t2[NB][CHh];
      hidden(l, y, t2, sBiasOdd, sBiasEven);
      if (l + 1 < L) {
        hidden(l + 1, t2, y, sBiasEven, sBiasOdd);
      } else {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int c = 0; c < CHh; ++c) y[nb][c] = t2[nb][c];
      }
    }
    // ---- output unit (Appendix B item 4) with the configured output map
    float zo[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) zo[nb] = 0.f;
    const float* wop = sWo + z + hf * (H / 2);
#pragma unroll
    for (int c = 0; c < CHh; ++c) {
#pragma unroll
      for (int e = 0; e < VPC; ++e) {
        const float wv = wop[VPC * c + e];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) zo[nb] += wv * T::get(y[nb][c], e);
      }
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) zo[nb] += __shfl_xor(zo[nb], 32) + bo;

    if (FWD_PART) {
      // ---- segmented ray-sum (Eq. (1)): scan within the tile, partials out
      const QueryDesc* qd = QUERY ? &a.qdesc[a.qtiles[t].slot] : nullptr;
      const bool slice = QUERY && qd->kind == 0;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float z = zo[nb];
        const float M = a.out_act ? fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))) : z;
        if (hf == 0) {
          const int tp = w * (NB * 32) + nb * 32 + pl;
          if (slice) {
            if (rid[nb] >= 0) qd->out[rid[nb]] = a.geom.mu0 * M;  // mu0 M: attenuation
            srid[tp] = -1;
          } else {
            sval[tp] = rid[nb] >= 0 ? M : 0.f;
            srid[tp] = rid[nb];
            if (QUERY) swgt[tp] = wgt[nb];
          }
        }
      }
      __syncthreads();
      const int tp = threadIdx.x;
      for (int o = 1; o < TILE; o <<= 1) {
        float add = 0.f;
        if (tp < TILE && tp >= o && srid[tp - o] == srid[tp]) add = sval[tp - o];
        __syncthreads();
        if (tp < TILE) sval[tp] += add;
        __syncthreads();
      }
      if (tp < TILE) {
        const int r = srid[tp];
        if (r >= 0 && (tp == TILE - 1 || srid[tp + 1] != r)) {
          const int64_t o0 = QUERY ? 0 : a.off[r];
          const int64_t o1 = QUERY ? 0 : a.off[r + 1];
          const int64_t tb = t * TILE;
          const float sum = sval[tp];
          if (QUERY) {
            // whole rays per tile: ray rid of this tile
            const QueryTile qt = a.qtiles[t];
            const int64_t ray = (int64_t)qt.tile * (TILE / qd->samples) + r;
            qd->out[ray] = __fmul_rn(swgt[tp], sum);
          } else if (MODE == MODE_FUSED) {
            // whole ray in this tile: prediction, residual, upstream gradient
            // rounded product (no contraction into the residual), as in the
            // forward kernel, so both passes produce the same residuals
            const float pbar = __fmul_rn(a.rays[r].wgt, sum);
            a.proj[r] = pbar;
            const float e = pbar - a.meas[r];
            lossacc += (double)e * (double)e;
            sg[o0 - tb] = g_scale * e;
          } else if (o0 < tb) {
            a.part[2 * t + 0] = sum;
          } else if (o1 > tb + TILE) {
            a.part[2 * t + 1] = sum;
          } else {
            a.proj[r] = __fmul_rn(a.rays[r].wgt, sum);
          }
        }
      }
      __syncthreads();
    }
    if (BWD_PART) {
      // ---- adjoint (Eq. (8)): dL/dM = g_r mu0 l_r / n_r, through the output map
      float dob[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float z = zo[nb];
        const float dMdz = a.out_act ? 1.f / (1.f + expf(-z)) : 1.f;
        float gr = 0.f;
        if (rid[nb] >= 0) gr = MODE == MODE_FUSED ? sg[poff[nb]] : a.gup[rid[nb]];
        dob[nb] = gr * wgt[nb] * dMdz;
      }
      // output-layer gradient: dw_o = sum_p dob_p h_L,p ; db_o = sum_p dob_p.
      // Halving butterfly over the 32 lanes of each half, in two passes over
      // the slots: after 5 steps lane pl holds the sums of KF consecutive slots.
      {
        constexpr int K = 32;  // slots per pass (the butterfly needs a multiple of 32)
#pragma unroll
        for (int pass = 0; pass < (H / 2) / K; ++pass) {
          float v[K];
#pragma unroll
          for (int i = 0; i < K; ++i) {
            const int rho = pass * K + i;
            float s = 0.f;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) s += dob[nb] * T::get(y[nb][rho / VPC], rho % VPC);
            v[i] = s;
          }
#pragma unroll
          for (int st = 0; st < 5; ++st) {
            const int o = 16 >> st;
            const int half = K >> (st + 1);
            const bool up = (pl & o) != 0;
#pragma unroll
            for (int i = 0; i < half; ++i) {
              const float send = up ? v[i] : v[i + half];
              const float keep = up ? v[i + half] : v[i];
              v[i] = keep + __shfl_xor(send, o);
            }
          }
          constexpr int KF = K / 32;
#pragma unroll
          for (int i = 0; i < KF; ++i) sdwo[w][feat(pass * K + KF * pl + i, hf)] += v[i];
        }
        float sb = 0.f;
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) sb += dob[nb];
#pragma unroll
        for (int o = 16; o > 0; o >>= 1) sb += __shfl_xor(sb, o);
        if (lane == 0) sdwo[w][H] += sb;
      }
      // delta_L = w_o dob . act'(z_L)
      chunk_t d[NB][CHh];
      if (ACT == 1) {
        // Swish: the last layer's derivatives, just stored by this wave
        wait_vm<0>();
        const char* ap = (const char*)astash(L - 1) + lane_off((uint32_t)(lane * sizeof(chunk_t)));
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int c = 0; c < CHh; ++c)
            d[nb][c] = *(const chunk_t*)(ap + (nb * CHh + c) * 64 * sizeof(chunk_t));
      }
#pragma unroll
      for (int c = 0; c < CHh; ++c) {
        float wv[VPC];
#pragma unroll
        for (int e = 0; e < VPC; ++e) wv[e] = wop[VPC * c + e];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          float v[VPC];
          if (ACT == 1) {
#pragma unroll
            for (int e = 0; e < VPC; ++e) v[e] = (wv[e] * dob[nb]) * T::get(d[nb][c], e);
          } else {
#pragma unroll
            for (int e = 0; e < VPC; ++e) {
              // h_L >= 0 (ReLU output): h > 0 iff its bit pattern is non-zero
              const int hb = __float_as_int(T::get(y[nb][c], e));
              const int keep = (int)neg_u32((uint32_t)hb) >> 31;  // 0 or all ones
              v[e] = __int_as_float(__float_as_int(wv[e] * dob[nb]) & keep);
            }
          }
          d[nb][c] = T::from_f32(v);
        }
      }
      auto dstash = [&](int l) { return (chunk_t*)a.stash + a.d_base[l] + blk0 * (CHh * 64); };
      if (L == 1) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int c = 0; c < CHh; ++c)
            T::store_nt(&dstash(0)[(nb * CHh + c) * 64 + lane], d[nb][c]);
      }
      // delta_{l-1} = (W_l^T delta_l) . relu'(z_{l-1}),  l = L .. 2; the layer
      // call stores its input delta_l for the weight gradient.  Two layers per
      // iteration with swapped roles, as in the forward.
      auto adj = [&](int l, const chunk_t (&in)[NB][CHh], chunk_t (&out)[NB][CHh]) {
        uint32_t mk[MSK_PER_LAYER];
        if (ACT == 0)
#pragma unroll
          for (int k = 0; k < MSK_PER_LAYER; ++k)
            mk[k] = msk_w[((l - 1) * MSK_PER_LAYER + k) * 64 + lane];
        const WSrc nx = l > 1 ? WTl(l - 1) : (more ? Wl(0) : none);
        const int nxb = l > 1 ? PB_H : PB_IN;
        // entering from the forward's last layer or from the previous adjoint
        // layer: both stored their last panel's share of a width-H input
        layer<PREC, CHh, H, ADJ_EPI, NB * (CHh / (H / 32 / panel_obs<CHh, H>()))>(
            in, out, WTl(l), nx, nxb, nullptr, none, nullptr, mk, dstash(l), sW0, sW1, lane, w, z,
            astash(l - 1));
      };
      for (int l = L - 1; l >= 1; l -= 2) {
        chunk_t t2[NB][CHh];
        adj(l, d, t2);
        if (l - 1 >= 1) {
          adj(l - 1, t2, d);
        } else {
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int c = 0; c < CHh; ++c) d[nb][c] = t2[nb][c];
        }
      }
      if (L > 1) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int c = 0; c < CHh; ++c)
            T::store_nt(&dstash(0)[(nb * CHh + c) * 64 + lane], d[nb][c]);
      }
    }
  }
  wait_vm<0>();
  if (BWD_PART) {
    __syncthreads();
    for (int f = threadIdx.x; f <= H; f += blockDim.x) {
      float s = 0.f;
      for (int ww = 0; ww < WAVES_PER_WG; ++ww) s += sdwo[ww][f];
      a.opart[(int64_t)blockIdx.x * (H + 1) + f] = s;
    }
  }
  if (MODE == MODE_FUSED) {
    sloss[threadIdx.x] = lossacc;
    __syncthreads();
    for (int o = WAVES_PER_WG * 32; o > 0; o >>= 1) {
      if (threadIdx.x < o) sloss[threadIdx.x] += sloss[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.lpart[blockIdx.x] = sloss[0];
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

// Loss (Eq. (5)) in FP64 and the upstream gradient g_r = 2 (pbar_r - p_r) / R.
// One workgroup, fixed summation order.
__global__ __launch_bounds__(1024) void k_loss(const float* __restrict__ proj,
                                                const float* __restrict__ meas, int64_t R,
                                                float* __restrict__ g, double* __restrict__ loss) {
  __shared__ double s[1024];
  const int t = threadIdx.x;
  double acc = 0.0;
  const float inv = 2.0f / (float)R;
  for (int64_t r = t; r < R; r += 1024) {
    const float e = proj[r] - meas[r];
    acc += (double)e * (double)e;
    g[r] = inv * e;
  }
  s[t] = acc;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) s[t] += s[t + o];
    __syncthreads();
  }
  if (t == 0) *loss = s[0] / (double)R;
}

// Loss of the fused pass: the MLP kernel's per-workgroup sums of squared
// residuals, plus rays that hold no samples (prediction 0, so the residual
// is the measurement) and rays with an invalid index (NaN).  One workgroup,
// fixed order.
__global__ __launch_bounds__(1024) void k_loss_fused(const RayRec* __restrict__ rays,
                                                      const float* __restrict__ meas, int64_t R,
                                                      const double* __restrict__ lpart,
                                                      int64_t n_lpart, float* __restrict__ proj,
                                                      double* __restrict__ loss) {
  __shared__ double s[1024];
  const int t = threadIdx.x;
  double acc = 0.0;
  for (int64_t k = t; k < n_lpart; k += 1024) acc += lpart[k];
  for (int64_t r = t; r < R; r += 1024) {
    const RayRec rr = rays[r];
    if (rr.flags & 1) {
      proj[r] = __builtin_nanf("");
      acc += (double)__builtin_nanf("");
    } else if (rr.n == 0) {
      proj[r] = 0.f;
      acc += (double)meas[r] * (double)meas[r];
    }
  }
  s[t] = acc;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (t < o) s[t] += s[t + o];
    __syncthreads();
  }
  if (t == 0) *loss = s[0] / (double)R;
}

// ------------------------------------------------------------ dW

// dW_l[o][i] = sum_p delta_l[p][o] h_{l-1}[p][i]  (and db_l = sum_p delta_l[p])
// over the stash blocks of one split.  The stash holds blocks of 32 points in
// the register layout of k_mlp; each iteration transposes NBLK blocks through
// LDS into [feature][point] rows so that both matrix-core operands are read
// as 16-byte runs of consecutive points (K = points).  The stash chunks of the
// next iteration are loaded into registers while the current one is reduced.
// COORDS: the h blocks hold point coordinates (layer 1) and the encoding is
// re-derived; otherwise they hold h_{l-1} in the register-chunk layout.
// Threads per weight-gradient workgroup: 16 waves at H = 256 (four per SIMD,
// each holding a quarter of the 32x32 output tiles, so that twice as many
// stash loads are in flight per compute unit as with 8 waves), 8 below.
template <int H>
__host__ __device__ constexpr int wgrad_threads() { return H >= 256 ? 1024 : 512; }

template <int PREC, int FI, int H, bool COORDS>
__global__ __launch_bounds__(wgrad_threads<H>()) void k_wgrad(WgArgs a) {
  using T = Prec<PREC>;
  using E = typename T::elem_t;
  using chunk_t = typename T::chunk_t;
  constexpr int VPC = T::VPC;
  constexpr int NBLK = PREC == PREC_BF16 ? 2 : 1;  // 32-point blocks per iteration
  constexpr int BP = 32 * NBLK;                     // points per iteration
  static_assert(Prec<PREC>::WAVES * Prec<PREC>::NB % (2 * NBLK) == 0,
                "a tile holds an even number of whole iterations");
  constexpr int CHd = chunks<PREC>(H), CHi = chunks<PREC>(FI);
  constexpr int ROW = BP + 16 / (int)sizeof(E);  // padded row (elements)
  constexpr int RB = H / 32, CB = FI / 32, NT = RB * CB;
  constexpr int NTH = wgrad_threads<H>();
  constexpr int NW = NTH / 64;
  constexpr int TPW = (NT + NW - 1) / NW;
  constexpr int QD = NBLK * CHd * 64 / NTH, QH = NBLK * CHi * 64 / NTH;  // chunks per thread
  static_assert(QD * NTH == NBLK * CHd * 64 && QH * NTH == NBLK * CHi * 64, "chunk split");
  // two buffer pairs of transposed operands ([feature][point] rows)
  __shared__ __align__(16) E sD0[H * ROW];
  __shared__ __align__(16) E sH0[FI * ROW];
  __shared__ __align__(16) E sD1[H * ROW];
  __shared__ __align__(16) E sH1[FI * ROW];
  __shared__ float4 sBr[FI / 2];  // GRFF rows when the h blocks hold coordinates
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, hf = lane >> 5;
  constexpr int G = NTH / BP;  // threads per point when encoding coordinates
  static_assert((FI / 2) % G == 0, "encoding rows split evenly over the point's threads");
  constexpr bool coords = COORDS;
  if (coords)
    for (int k = tid; k < FI / 2; k += blockDim.x) sBr[k] = a.Bmat[k];

  const int64_t P = a.off[a.R];
  const int64_t n_tiles = (P + a.tile - 1) / a.tile;
  int64_t pend = n_tiles * a.tile;
  if (pend > a.chunk_p1) pend = a.chunk_p1;
  const int64_t nblk = (pend - a.chunk_p0) / 32;  // valid 32-point blocks of the chunk
  const int64_t it0 = (int64_t)blockIdx.x * (a.kb / NBLK);
  int64_t it1 = it0 + a.kb / NBLK;
  const int64_t nit = (nblk + NBLK - 1) / NBLK;
  if (it1 > nit) it1 = nit;
  if (it0 >= it1) return;

  // tile k of wave w: 2 x 2 blocks of 32x32 tiles when the output divides
  // that way (each row and column fragment then serves two tiles), else a
  // strided walk over the tiles
  constexpr bool BLK2 = TPW == 4 && NW * 4 == NT && RB % 2 == 0 && CB % 2 == 0;
  auto tile_rc = [&](int k, int& rb, int& cb) -> bool {
    if (BLK2) {
      rb = 2 * (w / (CB / 2)) + (k >> 1);
      cb = 2 * (w % (CB / 2)) + (k & 1);
      return true;
    }
    const int tix = w + NW * k;
    rb = tix / CB;
    cb = tix % CB;
    return tix < NT;
  };
  f32x16 acc[TPW];
#pragma unroll
  for (int k = 0; k < TPW; ++k)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[k][r] = 0.f;
  float dbacc = 0.f;

  const chunk_t* __restrict__ Dst = (const chunk_t*)a.stash + a.d_base;
  const chunk_t* __restrict__ Hst = (const chunk_t*)a.stash + a.h_base;
  const float4* __restrict__ Cst = (const float4*)a.stash + a.h_base;
  chunk_t cd[QD], ch[QH];
  float4 rc;  // coordinates of point tid % BP (coordinate mode)
  // Addresses: a uniform base per iteration plus a 32-bit per-thread byte
  // offset (kept opaque so it is not widened into 64-bit addresses that are
  // hoisted, spilled and reloaded between the prefetch loads).
  const uint32_t toff = lane_off((uint32_t)tid * (uint32_t)sizeof(chunk_t));
  auto load = [&](int64_t it, chunk_t (&d)[QD], chunk_t (&h)[QH], float4& r) {
    const char* db = (const char*)(Dst + it * (NBLK * CHd * 64));
#pragma unroll
    for (int k = 0; k < QD; ++k) {
      const int q = tid + NTH * k;
      const bool ok = it * NBLK + q / (CHd * 64) < nblk;
      d[k] = ok ? *(const chunk_t*)(db + toff + NTH * k * sizeof(chunk_t)) : T::zero();
    }
    if (coords) {
      const int p = tid % BP;
      r = it * NBLK + p / 32 < nblk ? Cst[it * BP + p] : make_float4(0.f, 0.f, 0.f, 0.f);
      return;
    }
    const char* hb = (const char*)(Hst + it * (NBLK * CHi * 64));
#pragma unroll
    for (int k = 0; k < QH; ++k) {
      const int q = tid + NTH * k;
      const bool ok = it * NBLK + q / (CHi * 64) < nblk;
      h[k] = ok ? *(const chunk_t*)(hb + toff + NTH * k * sizeof(chunk_t)) : T::zero();
    }
  };
  // Transposition of the registers' iteration into one LDS buffer pair, and
  // the weight-gradient MFMAs over the other: the two buffers alternate, so
  // one iteration's transposition overlaps the previous one's MFMAs and each
  // iteration needs a single barrier.
  auto transpose = [&](E* tD, E* tH) {
#pragma unroll
    for (int k = 0; k < QD; ++k) {
      const int q = tid + NTH * k;
      const int bl = q / (CHd * 64), c = (q / 64) % CHd, l = q & 63;
      const int p = bl * 32 + (l & 31);
#pragma unroll
      for (int e = 0; e < VPC; ++e) tD[feat(VPC * c + e, l >> 5) * ROW + p] = (E)T::get(cd[k], e);
    }
    if (coords) {
      // layer 1's input h_0 = [cos 2 pi u ; sin 2 pi u] re-derived exactly as
      // the forward computed it (App. B item 2)
      const int p = tid % BP;
#pragma unroll 4
      for (int j = tid / BP; j < FI / 2; j += G) {
        float sv, cv;
        sincos_rev<PREC>(grff_phase(sBr[j], rc.x, rc.y, rc.z, rc.w), &sv, &cv);
        tH[j * ROW + p] = (E)cv;
        tH[(FI / 2 + j) * ROW + p] = (E)sv;
      }
    } else {
#pragma unroll
      for (int k = 0; k < QH; ++k) {
        const int q = tid + NTH * k;
        const int bl = q / (CHi * 64), c = (q / 64) % CHi, l = q & 63;
        const int p = bl * 32 + (l & 31);
#pragma unroll
        for (int e = 0; e < VPC; ++e) tH[feat(VPC * c + e, l >> 5) * ROW + p] = (E)T::get(ch[k], e);
      }
    }
  };
  auto contract = [&](const E* tD, const E* tH) {
    if (tid < H) {
      float sb = 0.f;
#pragma unroll
      for (int p = 0; p < BP; ++p) sb += (float)tD[tid * ROW + p];
      dbacc += sb;
    }
    // K-step outer, tiles inner: a wave's tiles share their row and column
    // fragments (2 x 2 blocks), which are read from LDS once per step
    constexpr int KS = PREC == PREC_BF16 ? BP / 16 : 4;
#pragma unroll
    for (int st = 0; st < KS; ++st) {
#pragma unroll
      for (int k = 0; k < TPW; ++k) {
        int rb, cb;
        if (tile_rc(k, rb, cb)) {
          const E* ra = tD + (32 * rb + (lane & 31)) * ROW;
          const E* rbp = tH + (32 * cb + (lane & 31)) * ROW;
          const int o = PREC == PREC_BF16 ? 16 * st + 8 * hf : 16 * hf + 4 * st;
          T::mma(acc[k], *(const chunk_t*)(ra + o), *(const chunk_t*)(rbp + o));
        }
      }
    }
  };
  auto clamp_it = [&](int64_t i) { return i < it1 ? i : it1 - 1; };
  load(it0, cd, ch, rc);
  transpose(sD0, sH0);
  load(clamp_it(it0 + 1), cd, ch, rc);
  __syncthreads();
  // a split's iteration count is even (whole tiles of an even number of
  // iterations, splits of a.kb / NBLK iterations), so the buffers alternate
  // in a fixed pattern
  for (int64_t it = it0; it < it1; it += 2) {
    transpose(sD1, sH1);  // iteration it + 1 (always within the split)
    load(clamp_it(it + 2), cd, ch, rc);
    contract(sD0, sH0);  // iteration it
    __syncthreads();
    if (it + 2 < it1) {
      transpose(sD0, sH0);  // iteration it + 2
      load(clamp_it(it + 3), cd, ch, rc);
    }
    contract(sD1, sH1);  // iteration it + 1
    __syncthreads();
  }
  // partial row of this split: same layout as the hidden part of the gradient
  float* out = a.wpart + (a.split_base + blockIdx.x) * a.nh;
#pragma unroll
  for (int k = 0; k < TPW; ++k) {
    int rb, cb;
    if (tile_rc(k, rb, cb)) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * rb + 8 * (r / 4) + 4 * hf + (r % 4);
        out[a.w_off + (int64_t)row * FI + 32 * cb + (lane & 31)] = acc[k][r];
      }
    }
  }
  if (tid < H) out[a.b_off + tid] = dbacc;
}

// grad[k] = compensated sum over valid split partials (hidden layers) or over
// the per-workgroup output-layer partials; per-block FP64 sums of grad^2.
__global__ __launch_bounds__(256) void k_reduce(RedArgs a) {
  __shared__ double s[256];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double sq = 0.0;
  if (k < a.np) {
    float sum = 0.f, comp = 0.f;
    if (k < a.nh) {
      const int64_t P = a.off[a.R];
      const int64_t n_tiles = (P + a.tile - 1) / a.tile;
      const int64_t pend = n_tiles * a.tile;
      for (int64_t c = 0; c < a.n_chunks; ++c) {
        const int64_t p0 = c * a.chunk_points;
        if (p0 >= pend) break;
        const int64_t pe = (pend < p0 + a.chunk_points) ? pend : p0 + a.chunk_points;
        const int64_t nblk = (pe - p0) / 32;
        const int64_t nsp = (nblk + a.kb - 1) / a.kb;
        for (int64_t i = 0; i < nsp; ++i) {
          const float y = a.wpart[(c * a.splits_per_chunk + i) * a.nh + k] - comp;
          const float t = sum + y;
          comp = (t - sum) - y;
          sum = t;
        }
      }
    } else {
      const int64_t j = k - a.nh;
      for (int64_t i = 0; i < a.n_opart; ++i) {
        const float y = a.opart[i * a.no + j] - comp;
        const float t = sum + y;
        comp = (t - sum) - y;
        sum = t;
      }
    }
    a.grad[k] = sum;
    sq = (double)sum * (double)sum;
  }
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

hipError_t launch_rays(const GeomDev& g, const int64_t* idx, int64_t R, RayRec* rays, int32_t* nray,
                       int32_t* n_out, int64_t* off, int tile, int64_t n_tiles_max, int32_t* tr0,
                       hipStream_t st) {
  const int bs = 256;
  const int64_t n_rec = R * g.sub * g.sub;  // ray records
  if (R > 0)
    hipLaunchKernelGGL(k_rays, dim3((unsigned)((R + bs - 1) / bs)), dim3(bs), 0, st, g, idx, R, rays,
                       nray, n_out);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, nray, n_rec, off);
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

template <int PREC, int IN, int H>
static hipError_t mlp_impl(int mode, const MlpArgs& a, int grid, hipStream_t st) {
  const dim3 b(Prec<PREC>::WAVES * 64);
  if (mode == MODE_FWD && a.act == 0)
    hipLaunchKernelGGL((k_mlp<PREC, IN, H, MODE_FWD, 0>), dim3(grid), b, 0, st, a);
  else if (mode == MODE_FWD)
    hipLaunchKernelGGL((k_mlp<PREC, IN, H, MODE_FWD, 1>), dim3(grid), b, 0, st, a);
  else if (mode == MODE_BWD && a.act == 0)
    hipLaunchKernelGGL((k_mlp<PREC, IN, H, MODE_BWD, 0>), dim3(grid), b, 0, st, a);
  else if (mode == MODE_BWD)
    hipLaunchKernelGGL((k_mlp<PREC, IN, H, MODE_BWD, 1>), dim3(grid), b, 0, st, a);
  else if (a.act == 0)
    hipLaunchKernelGGL((k_mlp<PREC, IN, H, MODE_FUSED, 0>), dim3(grid), b, 0, st, a);
  else
    hipLaunchKernelGGL((k_mlp<PREC, IN, H, MODE_FUSED, 1>), dim3(grid), b, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_mlp(int prec, int in, int h, int mode, const MlpArgs& a, int grid,
                      hipStream_t st) {
#define X(I, HH)                                                                   \
  if (in == I && h == HH)                                                          \
    return prec == PREC_BF16 ? mlp_impl<PREC_BF16, I, HH>(mode, a, grid, st)       \
                             : mlp_impl<PREC_F32, I, HH>(mode, a, grid, st);
  DINR_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

template <int PREC, int IN, int H>
static hipError_t query_impl(const MlpArgs& a, int grid, hipStream_t st) {
  if (a.act == 0)
    hipLaunchKernelGGL((k_mlp<PREC, IN, H, MODE_QUERY, 0>), dim3(grid), dim3(Prec<PREC>::WAVES * 64),
                       0, st, a);
  else
    hipLaunchKernelGGL((k_mlp<PREC, IN, H, MODE_QUERY, 1>), dim3(grid), dim3(Prec<PREC>::WAVES * 64),
                       0, st, a);
  return hipGetLastError();
}

hipError_t launch_query(int prec, int in, int h, const MlpArgs& a, int grid, hipStream_t st) {
#define X(I, HH)                                                          \
  if (in == I && h == HH)                                                 \
    return prec == PREC_BF16 ? query_impl<PREC_BF16, I, HH>(a, grid, st)  \
                             : query_impl<PREC_F32, I, HH>(a, grid, st);
  DINR_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_fixup(const RayRec* rays, const int64_t* off, int64_t R, int tile,
                        const float* part, float* proj, hipStream_t st) {
  if (R == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fixup, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, st, rays, off, R, tile,
                     part, proj);
  return hipGetLastError();
}

hipError_t launch_loss(const float* proj, const float* meas, int64_t R, float* g, double* loss,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_loss, dim3(1), dim3(1024), 0, st, proj, meas, R, g, loss);
  return hipGetLastError();
}

hipError_t launch_loss_fused(const RayRec* rays, const float* meas, int64_t R, const double* lpart,
                             int64_t n_lpart, float* proj, double* loss, hipStream_t st) {
  hipLaunchKernelGGL(k_loss_fused, dim3(1), dim3(1024), 0, st, rays, meas, R, lpart, n_lpart, proj,
                     loss);
  return hipGetLastError();
}

template <int PREC, int FI, int H, bool COORDS>
static hipError_t wgrad_impl(const WgArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_wgrad<PREC, FI, H, COORDS>), dim3(grid), dim3(wgrad_threads<H>()), 0, st,
                     a);
  return hipGetLastError();
}

hipError_t launch_wgrad(int prec, int fi, int h, const WgArgs& a, int grid, hipStream_t st) {
#define X(I, HH)                                                                  \
  if (h == HH && fi == I && a.coords)                                             \
    return prec == PREC_BF16 ? wgrad_impl<PREC_BF16, I, HH, true>(a, grid, st)    \
                             : wgrad_impl<PREC_F32, I, HH, true>(a, grid, st);    \
  if (h == HH && fi == HH && !a.coords)                                           \
    return prec == PREC_BF16 ? wgrad_impl<PREC_BF16, HH, HH, false>(a, grid, st)  \
                             : wgrad_impl<PREC_F32, HH, HH, false>(a, grid, st);
  DINR_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_reduce(const RedArgs& a, double* gnorm_ws, double* gnorm_out, hipStream_t st) {
  const unsigned nblk = (unsigned)((a.np + 255) / 256);
  hipLaunchKernelGGL(k_reduce, dim3(nblk), dim3(256), 0, st, a);
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
