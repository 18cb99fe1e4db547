// dinr_dev.h -- device-side building blocks shared by the libdinr kernels.
//
// Register layout of activations ("lane <-> point").  A wave evaluates the
// network for NB blocks of 32 points.  In each block, lane l holds point
// l % 32; the two lane halves (hf = l / 32) hold complementary halves of the
// point's feature vector.  Register slot rho (0 .. F/2-1) of half hf holds
// feature
//      feat(rho, hf) = 32 (rho/16) + 8 ((rho%16)/4) + 4 hf + (rho%4),
// which is exactly where a 32x32 matrix-core result leaves output row
// 32 ob + i (i = 8 (r/4) + 4 hf + r%4, r = rho - 16 ob).  A layer's output can
// therefore be fed to the next layer as its B operand (K = features,
// N = points) without moving data between lanes; the weights (A operand) are
// packed on the device with the same feature permutation along K.
//
// Slots are grouped into 16-byte "chunks": 8 bf16 values (one
// v_mfma_f32_32x32x16_bf16 K-step) or 4 fp32 values (four
// v_mfma_f32_32x32x2_f32 K-steps).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dinr {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(8 * sizeof(float)))) float f32x8;

enum { PREC_F32 = 0, PREC_BF16 = 1 };

constexpr int WAVE = 64;

__host__ __device__ constexpr int feat(int rho, int hf) {
  return 32 * (rho / 16) + 8 * ((rho % 16) / 4) + 4 * hf + (rho % 4);
}

template <int PREC>
struct Prec;

template <>
struct Prec<PREC_BF16> {
  using chunk_t = bf16x8;
  using elem_t = __bf16;
  static constexpr int VPC = 8;    // values per chunk per lane
  static constexpr int NB = 1;     // 32-point blocks per wave
  static constexpr int WAVES = 8;  // waves per workgroup (two per SIMD)
  __device__ static inline void mma(f32x16& acc, const chunk_t& a, const chunk_t& b) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  __device__ static inline chunk_t from_f32(const float* v) {
    f32x8 t = {v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]};
    return __builtin_convertvector(t, bf16x8);  // round to nearest even
  }
  __device__ static inline float get(const chunk_t& c, int e) { return (float)c[e]; }
  __device__ static inline chunk_t zero() {
    f32x8 t = {0, 0, 0, 0, 0, 0, 0, 0};
    return __builtin_convertvector(t, bf16x8);
  }
  // streaming store (non-temporal: does not displace reused data in L2)
  __device__ static inline void store_nt(chunk_t* p, const chunk_t& v) {
    __builtin_nontemporal_store(v, p);
  }
  // streaming load (data read once: kept from displacing reused data in L2)
  __device__ static inline chunk_t load_nt(const chunk_t* p) {
    return __builtin_nontemporal_load(p);
  }
};

template <>
struct Prec<PREC_F32> {
  using chunk_t = float4;
  using elem_t = float;
  static constexpr int VPC = 4;
  static constexpr int NB = 1;
  static constexpr int WAVES = 4;
  __device__ static inline void mma(f32x16& acc, const chunk_t& a, const chunk_t& b) {
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.z, b.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.w, b.w, acc, 0, 0, 0);
  }
  __device__ static inline chunk_t from_f32(const float* v) {
    return make_float4(v[0], v[1], v[2], v[3]);
  }
  __device__ static inline float get(const chunk_t& c, int e) {
    return e == 0 ? c.x : e == 1 ? c.y : e == 2 ? c.z : c.w;
  }
  __device__ static inline chunk_t zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
  __device__ static inline void store_nt(chunk_t* p, const chunk_t& v) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 t = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(t, (f4*)p);
  }
  __device__ static inline chunk_t load_nt(const chunk_t* p) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 t = __builtin_nontemporal_load((const f4*)p);
    return make_float4(t.x, t.y, t.z, t.w);
  }
};

// chunks per lane for F features
template <int PREC>
__host__ __device__ constexpr int chunks(int F) {
  return F / (2 * (PREC == PREC_BF16 ? 8 : 4));
}

// Per-ray record written by the ray-setup kernel.  Coordinates are already
// normalised to [-1,1]: point j of the ray is  pbar + (s_in + (j+u_j) dl) dbar,
// u_j = 1/2 or a stratified random offset, and its normalised time is tn.
// wgt = mu0 l / |Phi| (Eq. (1), (2), Appendix A).  ctr1..ctr3: words 1-3 of
// the position generator's counter (ray k in its projection, projection
// index low and high word).
struct __align__(16) RayRec {
  float px, py, pz, s_in;
  float dx, dy, dz, dl;
  float tn, wgt;
  int32_t n;
  int32_t flags;  // 1: index out of range
  uint32_t ctr1, ctr2, ctr3, pad;
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32 x 32 -> 64-bit products with multipliers 0xD2511F53 and 0xCD9E8D57, the
// key advanced by 0x9E3779B9 and 0xBB67AE85 after every round.  Returns the
// first output word, the only one the sample offsets use.
__device__ inline uint32_t philox_word0(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, x0), lo0 = 0xD2511F53u * x0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, x2), lo1 = 0xCD9E8D57u * x2;
    x0 = hi1 ^ x1 ^ k0;
    x1 = lo1;
    x2 = hi0 ^ x3 ^ k1;
    x3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return x0;
}

}  // namespace dinr
