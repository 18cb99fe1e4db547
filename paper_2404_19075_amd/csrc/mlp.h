// mlp.h -- the fused MLP kernel k_mlp (forward, adjoint, fused one-pass and
// query modes) and the device building blocks it shares with the weight
// gradient: ray construction, Fourier phases, weight-panel DMA into LDS.
// Included by the translation units that instantiate it.
#pragma once

#include "dinr_dev.h"
#include "kernels.h"
#include "ray_dev.h"

namespace dinr {

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
// drain_entry: wait for every outstanding memory operation before the first
// panel (the layer before issued no stash stores after its last DMA).
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
                             typename Prec<PREC>::chunk_t* __restrict__ actp = nullptr,
                             bool drain_entry = false) {
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
  // BF16 ReLU layers issue the panel's stash stores spread over the K-steps of
  // its first block (2 % faster than a burst after the barrier); the Swish
  // layers, whose epilogues also store and load derivatives, keep the burst
  // (spreading there is 12 % slower), and so does FP32 (spreading makes it spill)
  constexpr bool SPREAD = PREC == PREC_BF16 && (EPI == EPI_RELU_MASK || EPI == EPI_MASK);
  const int hf = lane >> 5;
  if (EPI == EPI_RELU_MASK)
#pragma unroll
    for (int k = 0; k < mask_words<PREC, H>(); ++k) msk[k] = 0u;
  f32x16 accp[NB];
  // EPI_DERIV: derivative chunk k of an output block, loaded at the K-step
  // where chunk k of the block before is consumed (one block of latency);
  // streaming loads, so that the weight panels stay in L2
  chunk_t actk[NEPI];
  const char* ap = (const char*)actp + lane_off((uint32_t)(lane * sizeof(chunk_t)));
#pragma unroll
  for (int ob = 0; ob < OB; ++ob) {
    if (ob % OBP == 0) {
      const int pi = ob / OBP;
      // the panel DMA'd last is complete; stores issued after it may still drain
      // (a layer without a stash simply waits for everything outstanding)
      if (stash) {
        // drain_entry: the layer before stored nothing after its last DMA
        if (pi == 0 && drain_entry) wait_vm<0>();
        else if (pi == 0) wait_vm<VM_ENTRY>();
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
      if (stash && !SPREAD) {
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
      if (SPREAD && stash && ob % OBP == 0 && c % (KC / SPP) == 0) {
        // the panel's stash stores, one every KC / SPP K-steps of its first block
        const int cs = (ob / OBP) * SPP + c / (KC / SPP);
        char* sp = (char*)stash + lane_off((uint32_t)(lane * sizeof(chunk_t)));
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          T::store_nt((chunk_t*)(sp + (nb * KC + cs) * 64 * sizeof(chunk_t)), x[nb][cs]);
      }
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
            actk[k] = T::load_nt((const chunk_t*)(ap + ((k / CPO) * chunks<PREC>(H) + ob * CPO +
                                                        k % CPO) * 64 * sizeof(chunk_t)));
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
  __shared__ float scomp[TILE];  // rounding errors of the segmented scan (TwoSum)
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
  constexpr bool GROUP = MODE == MODE_GROUP;
  static_assert(!GROUP || ACT == 1, "the group mode reads the activation derivatives from the stash");
  // group mode: per-wave sums of wgt h_L over the group's tiles, each ray's
  // (sum, Kahan compensation) and the group's upstream gradient
  __shared__ float sU[GROUP ? WAVES_PER_WG : 1][H + 1];
  __shared__ float sray_s[GROUP ? 64 : 1];
  __shared__ float sray_c[GROUP ? 64 : 1];
  __shared__ float sgp;
  const int64_t P = QUERY ? 0 : a.off[a.R];
  const int64_t n_tiles = QUERY ? a.n_qtiles : (P + TILE - 1) / TILE;
  const int64_t t_end = QUERY ? n_tiles : (a.tile_end < n_tiles ? a.tile_end : n_tiles);
  const float bo = a.params[a.bo_off];
  const int L = a.L;
  constexpr bool FWD_PART = MODE != MODE_BWD;
  constexpr bool BWD_PART = MODE == MODE_BWD || MODE == MODE_FUSED || MODE == MODE_GROUP;
  // the adjoint needs the ReLU masks (or the Swish derivatives) of the
  // forward layers
  constexpr int FWD_EPI = ACT == 1 ? (BWD_PART ? EPI_SWISH_D : EPI_SWISH)
                                   : (BWD_PART ? EPI_RELU_MASK : EPI_RELU);
  constexpr int ADJ_EPI = ACT == 1 ? EPI_DERIV : EPI_MASK;
  double lossacc = 0.0;
  // dL/dpbar = g_scale (pbar - p), g_scale = 2 / (number of projections)
  const float g_scale = 2.0f / (float)(GROUP ? a.n_proj : a.R);
  const __amdgpu_buffer_rsrc_t rW = buffer_rsrc(a.Wpk, a.wpk_bytes);
  const __amdgpu_buffer_rsrc_t rWT = buffer_rsrc(a.WTpk, a.wtpk_bytes);
  const __amdgpu_buffer_rsrc_t rB = buffer_rsrc(a.bias, (int64_t)L * H * sizeof(float));
  constexpr int ES = sizeof(typename T::elem_t);
  auto Wl = [&](int l) { return WSrc{rW, (int)(a.wpk_off[l] * ES)}; };
  auto WTl = [&](int l) { return WSrc{rWT, (int)(a.wtpk_off[l] * ES)}; };
  const WSrc none{rW, -1};

  // work units: tiles, or groups of a.group_tiles tiles (the chunk bounds are
  // multiples of the group)
  const int64_t u_begin = QUERY ? 0 : (GROUP ? a.tile_begin / a.group_tiles : a.tile_begin);
  const int64_t u_end = GROUP ? t_end / a.group_tiles : t_end;
  const int64_t u0 = u_begin + blockIdx.x;
  if (u0 < u_end) dma_panel<WAVES_PER_WG>(Wl(0), sW0, PB_IN, w, lane);
  for (int k = threadIdx.x; k < C; k += blockDim.x) sB[k] = a.Bmat[k];
  for (int k = threadIdx.x; k < H; k += blockDim.x) {
    sBias0[k] = a.bias[k];
    sWo[k] = a.wo_perm[k];
  }
  if (MODE != MODE_FWD)
    for (int k = threadIdx.x; k < WAVES_PER_WG * (H + 1); k += blockDim.x) (&sdwo[0][0])[k] = 0.f;
  if (GROUP)
    for (int k = threadIdx.x; k < WAVES_PER_WG * (H + 1); k += blockDim.x) (&sU[0][0])[k] = 0.f;
  __syncthreads();

  if constexpr (GROUP) {
    // ---- stash addresses of a tile: its first 32-point block for this wave
    auto blk_of = [&](int64_t t) -> int64_t { return (t - a.tile_begin) * (TILE / 32) + w * NB; };
    // Swish derivatives of layer l's outputs, in the layout of the stash: the
    // last layer's per point, the others' in the workgroup's ring (one group)
    auto astash = [&](int64_t blk0, int l) -> chunk_t* {
      if (!(BWD_PART && ACT == 1)) return nullptr;
      const int64_t rb = l + 1 < L ? (int64_t)blockIdx.x * a.ring_blocks + blk0 % a.ring_blocks
                                   : blk0;
      return (chunk_t*)a.stash + a.a_base[l] + rb * (CHh * 64);
    };
    auto hstash = [&](int64_t blk0, int l, int ch) -> chunk_t* {
      return BWD_PART ? (chunk_t*)a.stash + a.h_base[l] + blk0 * (ch * 64) : nullptr;
    };
    auto dstash = [&](int64_t blk0, int l) {
      return (chunk_t*)a.stash + a.d_base[l] + blk0 * (CHh * 64);
    };
    uint32_t* msk_w = &smsk[w][0][0][0];
    // biases of layer l+1 (none after the last layer: layer 0's stay resident)
    auto bias_next = [&](int l) -> WSrc {
      return l + 1 < L ? WSrc{rB, (l + 1) * H * (int)sizeof(float)} : none;
    };

    // ---- forward of tile t: coordinates, Fourier features, hidden layers and
    // the output unit.  Leaves each point's ray (rid; poff, the ray's first
    // point relative to the tile; its weight), h_L and the output pre-activation.
    // after_fwd: the first weight panel that follows the last forward layer.
    auto forward = [&](int64_t t, int z, WSrc after_fwd, int after_fwd_bytes, int (&rid)[NB],
                       int (&poff)[NB], float (&wgt)[NB], chunk_t (&y)[NB][CHh], float (&zo)[NB]) {
      const int64_t blk0 = blk_of(t);
      chunk_t x0[NB][CI];
      // ---- coordinates and Fourier features (Appendix A, Appendix B items 1-2)
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
      // ---- hidden layers (Appendix B item 3)
      {
        uint32_t mk[MSK_PER_LAYER];
        const WSrc nx = L > 1 ? Wl(1) : after_fwd;
        const int nxb = L > 1 ? PB_H : after_fwd_bytes;
        layer<PREC, CI, H, FWD_EPI, 0>(x0, y, Wl(0), nx, nxb, sBias0, bias_next(0), sBiasOdd,
                                             mk, nullptr, sW0, sW1, lane, w, z, astash(blk0, 0));
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
                                                   hstash(blk0, l, CHh), sW0, sW1, lane, w, z, astash(blk0, l));
        else
          layer<PREC, CHh, H, FWD_EPI, VM_H>(in, out, Wl(l), nx, nxb, sb, bias_next(l), sbn, mk,
                                                   hstash(blk0, l, CHh), sW0, sW1, lane, w, z, astash(blk0, l));
        if (BWD_PART && ACT == 0 && l < L - 1)
#pragma unroll
          for (int k = 0; k < MSK_PER_LAYER; ++k) msk_w[(l * MSK_PER_LAYER + k) * 64 + lane] = mk[k];
        if (BWD_PART && ACT == 0 && l == L - 1) {
          // the last layer's mask words: its weight gradient rebuilds delta_L from
          // them and dL/dz_o instead of reading it from the stash
          static_assert(MSK_PER_LAYER <= 4, "one 16-byte chunk per lane");
          u32x4 mw = {0u, 0u, 0u, 0u};
#pragma unroll
          for (int k = 0; k < MSK_PER_LAYER; ++k) mw[k] = mk[k];
          __builtin_nontemporal_store(mw, (u32x4*)a.stash + a.m_base + blk0 * 64 + lane);
        }
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
    };

    // output-layer gradient: dw_o = sum_p dob_p h_L,p ; db_o = sum_p dob_p.
    // Halving butterfly over the 32 lanes of each half, in two passes over
    // the slots: after 5 steps lane pl holds the sums of KF consecutive slots.
    // (dst: this wave's row of an LDS array; dst[H] receives db_o)
    auto dwo_acc = [&](const float (&dob)[NB], const chunk_t (&y)[NB][CHh], float* dst) {
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
        for (int i = 0; i < KF; ++i) dst[feat(pass * K + KF * pl + i, hf)] += v[i];
      }
      float sb = 0.f;
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) sb += dob[nb];
#pragma unroll
      for (int o = 16; o > 0; o >>= 1) sb += __shfl_xor(sb, o);
      if (lane == 0) dst[H] += sb;
    };

    // ---- adjoint of tile t (Eq. (8)) from dL/dz_o of its points: delta_L, the
    // delta chain through the transposed layers, the operand stash.
    // after: the first weight panel that follows the last adjoint layer.
    auto adjoint = [&](int64_t t, int z, const float (&dob)[NB], const chunk_t (&y)[NB][CHh],
                       WSrc after, int after_bytes) {
      const int64_t blk0 = blk_of(t);
      const float* wop = sWo + z + hf * (H / 2);
      // dL/dz_o of every point: the last layer's weight gradient rebuilds
      // delta_L from it (L >= 2: delta_L itself is not stashed)
      if (L >= 2 && hf == 0)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          __builtin_nontemporal_store(
              dob[nb], (float*)((chunk_t*)a.stash + a.dob_base) + (blk0 + nb) * 32 + pl);
      // delta_L = w_o dob . act'(z_L)
      chunk_t d[NB][CHh];
      if (ACT == 1) {
        // Swish: the last layer's derivatives, just stored by this wave
        wait_vm<0>();
        const char* ap = (const char*)astash(blk0, L - 1) +
                         lane_off((uint32_t)(lane * sizeof(chunk_t)));
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int c = 0; c < CHh; ++c)
            d[nb][c] =
                T::load_nt((const chunk_t*)(ap + (nb * CHh + c) * 64 * sizeof(chunk_t)));
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
      if (L == 1) {
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int c = 0; c < CHh; ++c)
            T::store_nt(&dstash(blk0, 0)[(nb * CHh + c) * 64 + lane], d[nb][c]);
      }
      // delta_{l-1} = (W_l^T delta_l) . relu'(z_{l-1}),  l = L .. 2; the layer
      // call stores its input delta_l for the weight gradient (but delta_L,
      // which the weight gradient rebuilds).  Two layers per iteration with
      // swapped roles, as in the forward.
      auto adj = [&](int l, const chunk_t (&in)[NB][CHh], chunk_t (&out)[NB][CHh]) {
        uint32_t mk[MSK_PER_LAYER];
        if (ACT == 0)
#pragma unroll
          for (int k = 0; k < MSK_PER_LAYER; ++k)
            mk[k] = msk_w[((l - 1) * MSK_PER_LAYER + k) * 64 + lane];
        const WSrc nx = l > 1 ? WTl(l - 1) : after;
        const int nxb = l > 1 ? PB_H : after_bytes;
        // entering from the forward's last layer or from the previous adjoint
        // layer: both stored their last panel's share of a width-H input
        layer<PREC, CHh, H, ADJ_EPI, NB * (CHh / (H / 32 / panel_obs<CHh, H>()))>(
            in, out, WTl(l), nx, nxb, nullptr, none, nullptr, mk,
            l == L - 1 ? nullptr : dstash(blk0, l), sW0, sW1, lane, w, z, astash(blk0, l - 1),
            l == L - 2);
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
            T::store_nt(&dstash(blk0, 0)[(nb * CHh + c) * 64 + lane], d[nb][c]);
      }
    };

    // Work units: tiles, or (group mode) groups of G consecutive tiles that
    // hold one projection each.
    const int G = GROUP ? a.group_tiles : 1;
    for (int64_t u = u0; u < u_end; u += gridDim.x) {
      const bool more = u + gridDim.x < u_end;
      for (int k = 0; k < G; ++k) {
        const int64_t t = u * G + k;
        // a zero the compiler cannot see through: keeps the per-lane loads of B
        // rows, biases and w_o inside the tile loop instead of hoisting (and
        // spilling) hundreds of loop-invariant values
        int z = 0;
        asm volatile("" : "+v"(z));
        int rid[NB];
        int poff[NB];
        float wgt[NB];
        chunk_t y[NB][CHh];
        float zo[NB];
        // what follows the last forward layer in the panel sequence: the
        // adjoint (its last layer's transposed weights) or the next tile; in
        // the group mode the next tile of the group until its last
        WSrc after_fwd = (BWD_PART && L > 1) ? WTl(L - 1) : (more ? Wl(0) : none);
        int after_fwd_bytes = (BWD_PART && L > 1) ? PB_H : PB_IN;
        if (GROUP && k + 1 < G) {
          after_fwd = Wl(0);
          after_fwd_bytes = PB_IN;
        }
        forward(t, z, after_fwd, after_fwd_bytes, rid, poff, wgt, y, zo);
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
                scomp[tp] = 0.f;
                srid[tp] = rid[nb];
                if (QUERY) swgt[tp] = wgt[nb];
              }
            }
          }
          __syncthreads();
          // inclusive scan of every ray's samples in the tile, compensated: each
          // step adds the partial o places back with TwoSum (Knuth) and carries
          // the rounding error, so a ray's sum is s + c with the error of a few
          // roundings whatever its number of samples and their magnitudes
          const int tp = threadIdx.x;
          for (int o = 1; o < TILE; o <<= 1) {
            float add = 0.f, addc = 0.f;
            if (tp < TILE && tp >= o && srid[tp - o] == srid[tp]) {
              add = sval[tp - o];
              addc = scomp[tp - o];
            }
            __syncthreads();
            if (tp < TILE) {
              const float x = sval[tp];
              const float s = x + add;
              const float bv = s - x;
              const float err = (x - (s - bv)) + (add - bv);
              sval[tp] = s;
              scomp[tp] = (scomp[tp] + addc) + err;
            }
            __syncthreads();
          }
          if (tp < TILE) {
            const int r = srid[tp];
            if (r >= 0 && (tp == TILE - 1 || srid[tp + 1] != r)) {
              const int64_t o0 = QUERY ? 0 : a.off[r];
              const int64_t o1 = QUERY ? 0 : a.off[r + 1];
              const int64_t tb = t * TILE;
              const float sum = sval[tp] + scomp[tp];
              if (GROUP) {
                // the tile lies inside one ray: its sum is added to the ray's,
                // Kahan in tile order as k_fixup adds a ray's tile partials
                const int kr = k / a.tiles_per_ray;
                if (k % a.tiles_per_ray == 0) {
                  sray_s[kr] = sum;
                  sray_c[kr] = 0.f;
                } else {
                  const float yv = sum - sray_c[kr];
                  const float tt = sray_s[kr] + yv;
                  sray_c[kr] = (tt - sray_s[kr]) - yv;
                  sray_s[kr] = tt;
                }
              } else if (QUERY) {
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
        if (GROUP) {
          // the group's dw_o is g_proj sum_k wgt_k sum_{p in tile k} h_L,p (a
          // linear output: dM/dz = 1); the weighted sum waits for g_proj
          dwo_acc(wgt, y, &sU[w][0]);
        }
      }
      if constexpr (GROUP) {
        // ---- the group's projection (Eq. (1), App. A): its rays' weighted sums
        // added in FP64 and rounded once, as k_bundle adds them; the residual,
        // its loss term and the upstream gradient 2 (pbar - p) / R (Eq. (5))
        if (threadIdx.x == 0) {
          const int64_t r = u;
          double acc = 0.0;
          bool bad = false;
          for (int kr = 0; kr < a.d2; ++kr) {
            const int64_t q = r * a.d2 + kr;
            bad = bad || (a.rays[q].flags & 1) != 0;
            acc += (double)__fmul_rn(a.rays[q].wgt, sray_s[kr]);
          }
          const float pbar = bad ? __builtin_nanf("") : (float)acc;
          a.proj[r] = pbar;
          const float e = pbar - a.meas[r];
          lossacc += (double)e * (double)e;
          sgp = g_scale * e;
        }
        __syncthreads();
        const float gp = sgp;
        for (int f = lane; f <= H; f += 64) {
          sdwo[w][f] += gp * sU[w][f];
          sU[w][f] = 0.f;
        }
        // ---- the adjoint of the group's tiles: every point of tile t belongs
        // to ray record t / m (m tiles per ray; a ray that misses the field of
        // view is padded to n points of weight 0)
        for (int k = 0; k < G; ++k) {
          const int64_t t = u * G + k;
          int z = 0;
          asm volatile("" : "+v"(z));
          const float wt = a.rays[t / a.tiles_per_ray].wgt;
          float dob[NB];
          chunk_t y[NB][CHh];  // h_L: the Swish adjoint does not read it
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) dob[nb] = gp * wt;
          const bool last = k + 1 == G;
          adjoint(t, z, dob, y, last ? (more ? Wl(0) : none) : WTl(L - 1), last ? PB_IN : PB_H);
        }
      }
    }
  } else {
    for (int64_t t = u0; t < t_end; t += gridDim.x) {
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
      // Swish derivatives of layer l's outputs, in the layout of the stash: the
      // last layer's per point, the others' in the workgroup's ring (one tile)
      auto astash = [&](int l) -> chunk_t* {
        if (!(BWD_PART && ACT == 1)) return nullptr;
        const int64_t rb =
            l + 1 < L ? (int64_t)blockIdx.x * a.ring_blocks + blk0 % a.ring_blocks : blk0;
        return (chunk_t*)a.stash + a.a_base[l] + rb * (CHh * 64);
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
        if (BWD_PART && ACT == 0 && l == L - 1) {
          // the last layer's mask words: its weight gradient rebuilds delta_L from
          // them and dL/dz_o instead of reading it from the stash
          static_assert(MSK_PER_LAYER <= 4, "one 16-byte chunk per lane");
          u32x4 mw = {0u, 0u, 0u, 0u};
#pragma unroll
          for (int k = 0; k < MSK_PER_LAYER; ++k) mw[k] = mk[k];
          __builtin_nontemporal_store(mw, (u32x4*)a.stash + a.m_base + blk0 * 64 + lane);
        }
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
              scomp[tp] = 0.f;
              srid[tp] = rid[nb];
              if (QUERY) swgt[tp] = wgt[nb];
            }
          }
        }
        __syncthreads();
        // inclusive scan of every ray's samples in the tile, compensated: each
        // step adds the partial o places back with TwoSum (Knuth) and carries
        // the rounding error, so a ray's sum is s + c with the error of a few
        // roundings whatever its number of samples and their magnitudes
        const int tp = threadIdx.x;
        for (int o = 1; o < TILE; o <<= 1) {
          float add = 0.f, addc = 0.f;
          if (tp < TILE && tp >= o && srid[tp - o] == srid[tp]) {
            add = sval[tp - o];
            addc = scomp[tp - o];
          }
          __syncthreads();
          if (tp < TILE) {
            const float x = sval[tp];
            const float s = x + add;
            const float bv = s - x;
            const float err = (x - (s - bv)) + (add - bv);
            sval[tp] = s;
            scomp[tp] = (scomp[tp] + addc) + err;
          }
          __syncthreads();
        }
        if (tp < TILE) {
          const int r = srid[tp];
          if (r >= 0 && (tp == TILE - 1 || srid[tp + 1] != r)) {
            const int64_t o0 = QUERY ? 0 : a.off[r];
            const int64_t o1 = QUERY ? 0 : a.off[r + 1];
            const int64_t tb = t * TILE;
            const float sum = sval[tp] + scomp[tp];
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
        // dL/dz_o of every point: the last layer's weight gradient rebuilds
        // delta_L from it (L >= 2: delta_L itself is not stashed)
        if (L >= 2 && hf == 0)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            __builtin_nontemporal_store(
                dob[nb], (float*)((chunk_t*)a.stash + a.dob_base) + (blk0 + nb) * 32 + pl);
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
              d[nb][c] =
                T::load_nt((const chunk_t*)(ap + (nb * CHh + c) * 64 * sizeof(chunk_t)));
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
        // call stores its input delta_l for the weight gradient (but delta_L,
        // which the weight gradient rebuilds).  Two layers per iteration with
        // swapped roles, as in the forward.
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
              in, out, WTl(l), nx, nxb, nullptr, none, nullptr, mk,
              l == L - 1 ? nullptr : dstash(l), sW0, sW1, lane, w, z, astash(l - 1), l == L - 2);
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
  if (MODE == MODE_FUSED || GROUP) {
    sloss[threadIdx.x] = lossacc;
    __syncthreads();
    for (int o = WAVES_PER_WG * 32; o > 0; o >>= 1) {
      if (threadIdx.x < o) sloss[threadIdx.x] += sloss[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.lpart[blockIdx.x] = sloss[0];
  }
}

// Launch of one instance (explicitly instantiated in mlp_inst.hip).
template <int PREC, int IN, int H, int MODE, int ACT>
hipError_t mlp_launch(const MlpArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_mlp<PREC, IN, H, MODE, ACT>), dim3(grid), dim3(Prec<PREC>::WAVES * 64), 0,
                     st, a);
  return hipGetLastError();
}

}  // namespace dinr
