// wgrad.hip -- weight-gradient reduction over the adjoint stash (k_wgrad).
#include "mlp.h"

namespace dinr {

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

// DM: 0 delta blocks from the stash; 1 the last layer's delta rebuilt from
// dL/dz_o and the ReLU mask words; 2 from dL/dz_o and the Swish derivatives.
// The last layer's delta is w_o[f] dL/dz_o act'(z_L)[f] (Eq. 5 through the
// linear output): the transposition forms dL/dz_o act'(z_L) and the factor
// w_o[f], common to row f of dW_L and to db_L[f], scales the finished rows.
template <int PREC, int FI, int H, bool COORDS, int DM>
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
  // the table is read by other threads in the first transposition
  __syncthreads();
  // rebuilt delta: the mask bits of the register slots rho = VPC c + e of a
  // thread's k-th chunk (q = tid + NTH k, c = (q / 64) mod CHd) sit at a place
  // that does not depend on the iteration, so it is set once; when NTH / 64 is
  // a multiple of CHd, c is the same for every k.  As the forward epilogue
  // records them (output block ob = rho / 16 owns bits of word ob / 2): BF16
  // word c / 4, bit 4 (c mod 4) + e / 2 + 16 (e mod 2); FP32 word c / 8, bit
  // 16 ((c / 4) mod 2) + 4 (c mod 4) + e.
  constexpr int NC = (NTH / 64) % CHd == 0 ? 1 : QD;
  int m_word[NC], m_shift[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int c = ((tid + NTH * k) / 64) % CHd;
    m_word[k] = PREC == PREC_BF16 ? c / 4 : c / 8;
    m_shift[k] = PREC == PREC_BF16 ? 4 * (c % 4) : 16 * ((c / 4) % 2) + 4 * (c % 4);
  }

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
  float dbacc = 0.f, dbcomp = 0.f;  // bias gradient of the split, Kahan-summed

  // delta blocks, or (rebuilt delta) the Swish derivative blocks / mask chunks
  const chunk_t* __restrict__ Dst =
      (const chunk_t*)a.stash + (DM == 2 ? a.m_base : DM == 1 ? a.m_base : a.d_base);
  const float* __restrict__ Dob = (const float*)((const chunk_t*)a.stash + a.dob_base);
  float dobv[DM ? QD : 1];
  uint32_t mw[DM == 1 ? QD : 1];
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
      const int64_t blk = it * NBLK + q / (CHd * 64);
      const bool ok = blk < nblk;
      if (DM == 1) {
        // the word of lane q % 64's mask chunk that holds this thread's slots
        // (shifted to bit 0), and the point's dL/dz_o
        const int kc = NC == 1 ? 0 : k;
        mw[k] = ok ? __builtin_nontemporal_load((const uint32_t*)(Dst + blk * 64 + (q & 63)) +
                                                m_word[kc]) >> m_shift[kc]
                   : 0u;
      } else {
        d[k] = ok ? T::load_nt((const chunk_t*)(db + toff + NTH * k * sizeof(chunk_t))) : T::zero();
      }
      if (DM) dobv[k] = ok ? __builtin_nontemporal_load(Dob + blk * 32 + (q & 31)) : 0.f;
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
      h[k] = ok ? T::load_nt((const chunk_t*)(hb + toff + NTH * k * sizeof(chunk_t))) : T::zero();
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
      // rebuilt delta: delta_L / w_o = dL/dz_o . act'(z_L); the factor w_o of
      // row f scales the finished row.  ReLU: the element is dL/dz_o where
      // the mask bit is set, else 0.  In BF16 the bits of slots 2j and 2j + 1
      // are bits j and j + 16 of the word, so (word >> j) & 0x10001 times the
      // 16 bits of dL/dz_o is the packed pair (one 24-bit multiply).
      if constexpr (DM == 1 && PREC == PREC_BF16) {
        const uint32_t dbits = __builtin_bit_cast(uint16_t, (E)dobv[k]);
#pragma unroll
        for (int j = 0; j < VPC / 2; ++j) {
          const uint32_t pr = ((mw[k] >> j) & 0x10001u) * dbits;
          tD[feat(VPC * c + 2 * j, l >> 5) * ROW + p] = __builtin_bit_cast(E, (uint16_t)pr);
          tD[feat(VPC * c + 2 * j + 1, l >> 5) * ROW + p] =
              __builtin_bit_cast(E, (uint16_t)(pr >> 16));
        }
        continue;
      }
      // Swish, BF16: the pair 2j, 2j + 1 is rounded by one packed conversion
      if constexpr (DM == 2 && PREC == PREC_BF16) {
        typedef __attribute__((__vector_size__(2 * sizeof(float)))) float f32x2_t;
        typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2_t;
#pragma unroll
        for (int j = 0; j < VPC / 2; ++j) {
          const f32x2_t v = {dobv[k] * T::get(cd[k], 2 * j), dobv[k] * T::get(cd[k], 2 * j + 1)};
          const bf16x2_t r = __builtin_convertvector(v, bf16x2_t);
          tD[feat(VPC * c + 2 * j, l >> 5) * ROW + p] = r[0];
          tD[feat(VPC * c + 2 * j + 1, l >> 5) * ROW + p] = r[1];
        }
        continue;
      }
#pragma unroll
      for (int e = 0; e < VPC; ++e) {
        const int f = feat(VPC * c + e, l >> 5);
        if (DM == 0) {
          tD[f * ROW + p] = (E)T::get(cd[k], e);
        } else if (DM == 2) {
          tD[f * ROW + p] = (E)(dobv[k] * T::get(cd[k], e));
        } else {
          tD[f * ROW + p] = ((mw[k] >> e) & 1u) ? (E)dobv[k] : (E)0.f;
        }
      }
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
      const float y = sb - dbcomp;
      const float t = dbacc + y;
      dbcomp = (t - dbacc) - y;
      dbacc = t;
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
        out[a.w_off + (int64_t)row * FI + 32 * cb + (lane & 31)] =
            DM ? acc[k][r] * a.wo[row] : acc[k][r];
      }
    }
  }
  if (tid < H) out[a.b_off + tid] = DM ? dbacc * a.wo[tid] : dbacc;
}

// dW_l and db_l of a BF16 layer of width 256 (fan-in 256): the same reduction
// as k_wgrad, with the stash streamed by DMA straight into an LDS ring of
// four 32-point blocks and the matrix-core operands read out of the ring with
// transposing loads (ds_read_b64_tr_b16) instead of being transposed element
// by element through registers.  Within a 16-lane group that load hands lane
// 4q + i element i of the 8-byte reads of lanes q, q + 4, q + 8, q + 12; a
// stash chunk's elements 4j .. 4j + 3 are four consecutive features of one
// point (feat()), so lanes q + 4e reading points p0 + e of the same four
// features give lane 4q + i feature i of them at four consecutive points: a
// quarter of its operand (rows = features, K = points).  Two such loads make
// the eight points of a 32x32x16 operand.  The ring keeps the chunk layout of
// the stash except that the upper half of each chunk (lanes 32-63) is stored
// at point index p xor 4, so that a group's eight 16-byte pieces fall in
// distinct LDS banks.
// DM 0: delta blocks copied from the stash (three blocks ahead).  DM 1 / 2:
// the last layer's delta / w_o = dL/dz_o . act'(z_L), built in the ring from
// the copied ReLU mask words or Swish derivatives and dL/dz_o, and w_o[f]
// scales the finished rows.  COORDS: h_0 is the Fourier encoding of the
// copied coordinates (App. B item 2), built in the ring through the forward's
// phase and sin/cos functions.  Blocks that are built are built one step
// ahead of their reduction (copies two blocks ahead).
constexpr int WTR_THREADS = 1024;

__device__ inline bf16x8 tr_pair(const char* a0, const char* a1) {
  typedef short v4i16 __attribute__((ext_vector_type(4)));
  typedef short v8i16 __attribute__((ext_vector_type(8)));
  const v4i16 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
      (__attribute__((address_space(3))) v4i16*)(const_cast<char*>(a0)));
  const v4i16 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
      (__attribute__((address_space(3))) v4i16*)(const_cast<char*>(a1)));
  const v8i16 v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  return __builtin_bit_cast(bf16x8, v);
}

// Wait until at most n vector-memory operations are outstanding (n < 16).
__device__ inline void wait_vm_n(int n) {
  switch (n) {
    case 0: wait_vm<0>(); break;
    case 1: wait_vm<1>(); break;
    case 2: wait_vm<2>(); break;
    case 3: wait_vm<3>(); break;
    case 4: wait_vm<4>(); break;
    case 5: wait_vm<5>(); break;
    default: wait_vm<6>(); break;
  }
}

template <int DM, bool COORDS>
__global__ __launch_bounds__(WTR_THREADS) void k_wgrad_tr(WgArgs a) {
  constexpr int H = 256, FI = 256, CH = H / 16;  // 16-byte chunks per lane and block
  constexpr int NW = WTR_THREADS / 64;           // 16 waves: wave w moves chunk w
  static_assert(NW == CH, "one delta and one h chunk per wave and block");
  static_assert(!(COORDS && DM != 0), "layer 1's delta is stashed");
  constexpr bool BUILD = DM != 0 || COORDS;
  constexpr int HALF = CH * 1024;                // delta (or h) bytes of one block
  constexpr int AUX = 2 * HALF;                  // mask words or coordinates (1 KB), dL/dz_o
  constexpr int SLOT = 2 * HALF + (BUILD ? 2048 : 0);
  __shared__ __align__(16) char ring0[SLOT];
  __shared__ __align__(16) char ring1[SLOT];
  __shared__ __align__(16) char ring2[SLOT];
  __shared__ __align__(16) char ring3[SLOT];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // COORDS: the GRFF rows of the four features this thread encodes, the same
  // for every block
  float4 brow[4];
  if (COORDS) {
    const int lam = (tid >> 1) & 63;
    const int L = lam < 32 ? lam : 32 + ((lam - 32) ^ 4);
#pragma unroll
    for (int i = 0; i < 4; ++i) brow[i] = a.Bmat[feat(8 * (tid >> 7) + 4 * (tid & 1) + i, L >> 5)];
  }

  const int64_t P = a.off[a.R];
  const int64_t n_tiles = (P + a.tile - 1) / a.tile;
  int64_t pend = n_tiles * a.tile;
  if (pend > a.chunk_p1) pend = a.chunk_p1;
  const int64_t nblk = (pend - a.chunk_p0) / 32;  // valid 32-point blocks of the chunk
  // the split's blocks, as k_wgrad takes them (pairs of blocks; a pair that
  // straddles the end of the chunk reads zeros for its second block)
  const int64_t b0 = (int64_t)blockIdx.x * a.kb;
  const int64_t nb2 = (nblk + 1) / 2 * 2;
  if (b0 >= nb2) return;
  const int64_t b1 = b0 + ((b0 + a.kb < nb2 ? a.kb : nb2 - b0) + 3) / 4 * 4;

  // Copies of block b into a ring slot.  Wave w: delta chunk w (DM 0), or the
  // Swish derivative chunk w (DM 2); h chunk w (not COORDS); wave 0 also the
  // mask words (DM 1) or the coordinates (COORDS), wave 1 dL/dz_o (DM 1, 2).
  // A chunk's lane l gets the stash piece pi(l) (pi: the upper half at point
  // xor 4, an involution).  Blocks past the chunk's end get an empty buffer
  // range: the copy writes zeros.  Cache policy 2: streaming, read once.
  const int piece = lane < 32 ? lane : 32 + ((lane - 32) ^ 4);
  const uint32_t voff = lane_off((uint32_t)((w * 64 + piece) * 16));
  const uint32_t voff16 = lane_off((uint32_t)(lane * 16)), voff4 = lane_off((uint32_t)(lane * 4));
  const char* stash = (const char*)a.stash;
  constexpr bool d_copy = DM != 1, h_copy = !COORDS;
  const bool aux0 = (DM == 1 || COORDS) && w == 0, aux1 = DM != 0 && w == 1;
  // Copies per block: N_MIN by the waves without an auxiliary copy, N_MIN + 1
  // by the one or two waves with one, issued in the order delta, h, aux.  The
  // waits below are compile-time constants, the same for every wave (a wait
  // chosen per wave at run time makes the compiler add waits of its own before
  // the operand reads).  Blocks of copies only (DM 0, no auxiliary copies):
  // before step b at most 2 N_MIN copies, blocks b + 1 and b + 2, are in
  // flight, so block b has landed.  Built blocks: at most N_MIN + 1, that is
  // block b + 2's copies and, in the waves with N_MIN copies, the last of
  // block b + 1's (h for DM 1 and 2, delta for COORDS: neither is read by
  // block b + 1's build), so that build finds its auxiliary copies and, DM 2,
  // the delta chunk it rescales in place (copied by the same wave), and block
  // b's copies have all landed.  Before the first build: at most 2 N_MIN, all
  // from blocks b0 + 1 and b0 + 2 in every wave, so block b0 has landed.
  constexpr int N_MIN = (d_copy ? 1 : 0) + (h_copy ? 1 : 0);
  constexpr int WAIT_STEP = BUILD ? N_MIN + 1 : 2 * N_MIN, WAIT_FIRST = 2 * N_MIN;
  auto dma = [&](int64_t b, char* slot) {
    const bool ok = b < nblk;
    if (d_copy) {
      const char* d = stash + ((DM == 2 ? a.m_base : a.d_base) + b * CH * 64) * 16;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(buffer_rsrc(d, ok ? HALF : 0),
                                               (lds_void*)(slot + w * 1024), 16, (int)voff, 0,
                                               0, 2);
    }
    if (h_copy) {
      const char* h = stash + (a.h_base + b * CH * 64) * 16;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(buffer_rsrc(h, ok ? HALF : 0),
                                               (lds_void*)(slot + HALF + w * 1024), 16,
                                               (int)voff, 0, 0, 2);
    }
    if (aux0) {
      // 64 mask chunks (one per lane of the block), or 32 points' coordinates
      const char* m = COORDS ? stash + (a.h_base + b * 32) * 16 : stash + (a.m_base + b * 64) * 16;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(buffer_rsrc(m, ok ? (COORDS ? 512 : 1024) : 0),
                                               (lds_void*)(slot + AUX), 16, (int)voff16, 0, 0,
                                               2);
    }
    if (aux1) {
      const char* o = stash + a.dob_base * 16 + b * 32 * 4;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(buffer_rsrc(o, ok ? 128 : 0),
                                               (lds_void*)(slot + AUX + 1024), 4, (int)voff4, 0,
                                               0, 2);
    }
  };

  // Operands built in a slot from the copied sources (all threads).
  auto build = [&](char* slot) {
    if constexpr (DM == 2) {
      // delta / w_o = dL/dz_o . swish'(z_L), rounded once, in place
      const int c = tid >> 6, lam = tid & 63;
      const int pnt = (lam < 32 ? lam : 32 + ((lam - 32) ^ 4)) & 31;
      const float dob = ((const float*)(slot + AUX + 1024))[pnt];
      bf16x8* q = (bf16x8*)(slot + c * 1024 + lam * 16);
      const bf16x8 sd = *q;
      typedef __attribute__((__vector_size__(2 * sizeof(float)))) float f32x2_t;
      typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2_t;
      bf16x8 r;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const f32x2_t v = {dob * (float)sd[2 * j], dob * (float)sd[2 * j + 1]};
        const bf16x2_t b2 = __builtin_convertvector(v, bf16x2_t);
        r[2 * j] = b2[0];
        r[2 * j + 1] = b2[1];
      }
      *q = r;
    } else if constexpr (DM == 1) {
      // delta / w_o = dL/dz_o where the mask bit is set: the bits of slots 2j
      // and 2j + 1 of chunk c are bits j and j + 16 of word c / 4 shifted by
      // 4 (c mod 4), so (word >> j) & 0x10001 times the 16 bits of dL/dz_o is
      // the packed pair
      const int c = tid >> 6, lam = tid & 63;
      const int L = lam < 32 ? lam : 32 + ((lam - 32) ^ 4);
      const float dob = ((const float*)(slot + AUX + 1024))[L & 31];
      const uint32_t dbits = __builtin_bit_cast(uint16_t, (__bf16)dob);
      const uint32_t mw = ((const uint32_t*)(slot + AUX + L * 16))[c / 4] >> (4 * (c % 4));
      u32x4 r;
#pragma unroll
      for (int j = 0; j < 4; ++j) r[j] = ((mw >> j) & 0x10001u) * dbits;
      *(u32x4*)(slot + c * 1024 + lam * 16) = r;
    }
    if constexpr (COORDS) {
      // h_0 = [cos 2 pi u ; sin 2 pi u]: thread (c, lam, half) makes elements
      // 4 half .. + 3 of cos chunk c < 8 and of sin chunk c + 8
      const int lam = (tid >> 1) & 63;
      const int L = lam < 32 ? lam : 32 + ((lam - 32) ^ 4);
      const int c = tid >> 7, half = tid & 1;
      const float4 rc = ((const float4*)(slot + AUX))[L & 31];
      typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4_t;
      bf16x4_t cv, sv;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float s_, c_;
        sincos_rev<PREC_BF16>(grff_phase(brow[i], rc.x, rc.y, rc.z, rc.w), &s_, &c_);
        cv[i] = (__bf16)c_;
        sv[i] = (__bf16)s_;
      }
      *(bf16x4_t*)(slot + HALF + c * 1024 + lam * 16 + 8 * half) = cv;
      *(bf16x4_t*)(slot + HALF + (c + 8) * 1024 + lam * 16 + 8 * half) = sv;
    }
  };

  // operand addresses: wave w holds tiles (rb, cb) for rb in {2 (w / 4), +1},
  // cb in {2 (w % 4), +1}.  Lane l as a source of the transposing load: group
  // g = l / 16, s = l % 16, point offset e = s / 4, quad q = s % 4; rows
  // 16 (g % 2) + 4 q .. + 3 of the tile are features of chunk 2 rb + g % 2,
  // half q % 2, elements 4 (q / 2) .. + 3; points 8 (g / 2) + e (+ 4 for the
  // second load, + 16 for the second K-step)
  const int g = lane >> 4, e = (lane >> 2) & 3, q = lane & 3;
  const int hfq = q & 1, pl = 8 * (g >> 1) + e;
  // piece of point pl (first load) and pl + 4 (second), upper half at xor 4
  const int pc0 = hfq ? 32 + (pl ^ 4) : pl;
  const int pc1 = hfq ? 32 + ((pl + 4) ^ 4) : pl + 4;
  const int lane_b0 = pc0 * 16 + 8 * (q >> 1), lane_b1 = pc1 * 16 + 8 * (q >> 1);
  const int rb0 = 2 * (w / 4), cb0 = 2 * (w % 4);
  // byte offsets inside a slot of the rows this lane sources for the first
  // row (column) block of the wave; the second block is two chunks (2 KB)
  // further, the second K-step 16 points (256 B) further
  const int oa0 = (int)lane_off((uint32_t)((2 * rb0 + (g & 1)) * 1024 + lane_b0));
  const int oa1 = (int)lane_off((uint32_t)((2 * rb0 + (g & 1)) * 1024 + lane_b1));
  const int ob0 = (int)lane_off((uint32_t)(HALF + (2 * cb0 + (g & 1)) * 1024 + lane_b0));
  const int ob1 = (int)lane_off((uint32_t)(HALF + (2 * cb0 + (g & 1)) * 1024 + lane_b1));
  // bias gradient: the waves with w % 4 = 0 hold the delta fragments of every
  // row block; lane l sums its eight points of feature 32 rb + l % 32 for each
  // K-step, Kahan-accumulates the block's sum, and the two K halves (lanes l
  // and l + 32) are added at the end
  const bool db_wave = (w & 3) == 0;

  f32x16 acc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[k][r] = 0.f;
  float dbacc[2] = {0.f, 0.f}, dbcomp[2] = {0.f, 0.f};

  // one block: copies of block b (copied blocks) or of b + 1 (built blocks)
  // are done, the barrier publishes them (and the block built last step) and
  // frees the slot of block b - 1; then the next copies, the next build, and
  // the reduction of block b
  auto step = [&](int64_t b, char* cur, char* nb, char* nxt) {
    wait_vm<WAIT_STEP>();
    panel_barrier();
    // the work every wave must finish before the next barrier runs at a raised
    // wave priority: the next copies (blocks of copies only) or the next build
    if (BUILD) {
      dma(b + 3, nxt);
      __builtin_amdgcn_s_setprio(2);
      build(nb);
      __builtin_amdgcn_s_setprio(0);
    } else {
      __builtin_amdgcn_s_setprio(2);
      dma(b + 3, nxt);
      __builtin_amdgcn_s_setprio(0);
    }
    float sbk[2] = {0.f, 0.f};
#pragma unroll
    for (int st = 0; st < 2; ++st) {
      bf16x8 fa[2], fh[2];
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        fa[k] = tr_pair(cur + oa0 + 2048 * k + 256 * st, cur + oa1 + 2048 * k + 256 * st);
        fh[k] = tr_pair(cur + ob0 + 2048 * k + 256 * st, cur + ob1 + 2048 * k + 256 * st);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k)
        acc[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[k >> 1], fh[k & 1], acc[k], 0, 0, 0);
      if (db_wave) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          float sb = 0.f;
#pragma unroll
          for (int i = 0; i < 8; ++i) sb += (float)fa[k][i];
          sbk[k] += sb;
        }
      }
    }
    if (db_wave) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const float y = sbk[k] - dbcomp[k];
        const float t = dbacc[k] + y;
        dbcomp[k] = (t - dbacc[k]) - y;
        dbacc[k] = t;
      }
    }
  };
  dma(b0, ring0);
  dma(b0 + 1, ring1);
  dma(b0 + 2, ring2);
  if (BUILD) {
    // the first block is built before the loop
    wait_vm<WAIT_FIRST>();
    panel_barrier();
    build(ring0);
  }
  // the ring turns in steps of four: the split's block count is rounded up to
  // a multiple of four (only the chunk's last split can need it; the blocks
  // added lie past the chunk's end, copy as zeros and add nothing), so every
  // pass of the loop runs all four steps and the compiler's wait for a slot's
  // copies at the top of the loop counts the copies issued after them
  for (int64_t b = b0; b < b1; b += 4) {
    step(b, ring0, ring1, ring3);
    step(b + 1, ring1, ring2, ring0);
    step(b + 2, ring2, ring3, ring1);
    step(b + 3, ring3, ring0, ring2);
  }
  // drain the copies issued past the split's end before the workgroup exits
  wait_vm<0>();

  float* out = a.wpart + (a.split_base + blockIdx.x) * a.nh;
  const int hf = lane >> 5;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int rb = rb0 + (k >> 1), cb = cb0 + (k & 1);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 32 * rb + 8 * (r / 4) + 4 * hf + (r % 4);
      out[a.w_off + (int64_t)row * FI + 32 * cb + (lane & 31)] =
          DM ? acc[k][r] * a.wo[row] : acc[k][r];
    }
  }
  if (db_wave) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      // the upper half's points of the same feature (lane + 32), compensation
      // included
      const float own = dbacc[k] - dbcomp[k];
      const float other = __shfl_xor(own, 32);
      const int f = 32 * (rb0 + k) + lane;
      if (lane < 32) out[a.b_off + f] = DM ? (own + other) * a.wo[f] : own + other;
    }
  }
}

#define DINR_SHAPES(X) X(128, 64) X(256, 256)

template <int PREC, int FI, int H, bool COORDS, int DM>
static hipError_t wgrad_impl(const WgArgs& a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((k_wgrad<PREC, FI, H, COORDS, DM>), dim3(grid), dim3(wgrad_threads<H>()), 0,
                     st, a);
  return hipGetLastError();
}

template <int PREC, int FI, int H>
static hipError_t wgrad_hidden(const WgArgs& a, int grid, hipStream_t st) {
  switch (a.dmode) {
    case 0: return wgrad_impl<PREC, FI, H, false, 0>(a, grid, st);
    case 1: return wgrad_impl<PREC, FI, H, false, 1>(a, grid, st);
    case 2: return wgrad_impl<PREC, FI, H, false, 2>(a, grid, st);
  }
  return hipErrorInvalidValue;
}

// Layer 1 (coordinates) always reads stashed delta blocks: its delta is the
// last layer's only when L = 1, and then it is stashed.
hipError_t launch_wgrad(int prec, int fi, int h, const WgArgs& a, int grid, hipStream_t st) {
  if (prec == PREC_BF16 && fi == 256 && h == 256) {
    if (a.coords && a.dmode == 0)
      hipLaunchKernelGGL((k_wgrad_tr<0, true>), dim3(grid), dim3(WTR_THREADS), 0, st, a);
    else if (!a.coords && a.dmode == 0)
      hipLaunchKernelGGL((k_wgrad_tr<0, false>), dim3(grid), dim3(WTR_THREADS), 0, st, a);
    else if (!a.coords && a.dmode == 1)
      hipLaunchKernelGGL((k_wgrad_tr<1, false>), dim3(grid), dim3(WTR_THREADS), 0, st, a);
    else if (!a.coords && a.dmode == 2)
      hipLaunchKernelGGL((k_wgrad_tr<2, false>), dim3(grid), dim3(WTR_THREADS), 0, st, a);
    else
      return hipErrorInvalidValue;
    return hipGetLastError();
  }
#define X(I, HH)                                                                  \
  if (h == HH && fi == I && a.coords && a.dmode == 0)                             \
    return prec == PREC_BF16 ? wgrad_impl<PREC_BF16, I, HH, true, 0>(a, grid, st) \
                             : wgrad_impl<PREC_F32, I, HH, true, 0>(a, grid, st); \
  if (h == HH && fi == HH && !a.coords)                                           \
    return prec == PREC_BF16 ? wgrad_hidden<PREC_BF16, HH, HH>(a, grid, st)       \
                             : wgrad_hidden<PREC_F32, HH, HH>(a, grid, st);
  DINR_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace dinr
