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
};

// chunks per lane for F features
template <int PREC>
__host__ __device__ constexpr int chunks(int F) {
  return F / (2 * (PREC == PREC_BF16 ? 8 : 4));
}

// Per-ray record written by the ray-setup kernel.  Coordinates are already
// normalised to [-1,1]: point j of the ray is  pbar + (s_in + (j+1/2) dl) dbar
// and its normalised time is tn.  wgt = mu0 l / n (Eq. (1), (2)).
struct __align__(16) RayRec {
  float px, py, pz, s_in;
  float dx, dy, dz, dl;
  float tn, wgt;
  int32_t n;
  int32_t flags;  // 1: index out of range
};

}  // namespace dinr
