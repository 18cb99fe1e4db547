// ctx.h -- the library context shared by the training entry points and the
// query server (internal; the public interface is include/dinr.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <vector>

#include "dinr.h"
#include "kernels.h"

using namespace dinr;

struct dinr_ctx {
  int device = 0;
  int n_cu = 0;
  dinr_geometry geom{};
  dinr_mlp mlp{};
  dinr_sampling samp{};
  uint32_t epoch = 0;  // second key word of the sample-position generator
  int IN = 0, H = 0, L = 0, prec = 0, tile = 0, nmax = 0;
  int64_t np = 0, nh = 0;
  std::vector<int64_t> w_off, b_off;
  int64_t wo_off = 0, bo_off = 0;
  // device tables
  float* d_cth = nullptr;
  float* d_sth = nullptr;
  float* d_tn = nullptr;
  float4* d_B = nullptr;
  // workspace arena
  char* arena = nullptr;
  size_t arena_size = 0;
  int32_t* d_status = nullptr;  // [0] Adam skipped (non-finite)
  double* d_scal = nullptr;     // [0] loss, [1] gnorm
  char err[512] = {0};
  GeomDev gd{};
  // optional per-kernel timing: event pairs recorded around launches
  struct Prof {
    bool on = false;
    std::vector<hipEvent_t> ev[DINR_PROF_KINDS][2];
    size_t used[DINR_PROF_KINDS] = {0};
  } prof;
};

// Record a start/stop event pair around one launch of kernel class k.
struct ProfScope {
  dinr_ctx* c;
  int k;
  hipStream_t st;
  bool active = false;
  ProfScope(dinr_ctx* c_, int k_, hipStream_t st_) : c(c_), k(k_), st(st_) {
    auto& p = c->prof;
    if (p.on && p.used[k] < p.ev[k][0].size()) {
      hipEventRecord(p.ev[k][0][p.used[k]], st);
      active = true;
    }
  }
  ~ProfScope() {
    if (active) {
      auto& p = c->prof;
      hipEventRecord(p.ev[k][1][p.used[k]], st);
      ++p.used[k];
    }
  }
};

inline int fail(dinr_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(c->err, sizeof(c->err), fmt, ap);
    va_end(ap);
  }
  return code;
}

#define HIPCHK(ctx, x)                                                              \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess)                                                           \
      return fail(ctx, DINR_EHIP, "%s failed: %s", #x, hipGetErrorString(e_));       \
  } while (0)


// Packing layout of the context's network (forward and transposed fragments).
inline PackArgs pack_layout(const dinr_ctx* c) {
  PackArgs k{};
  k.L = c->L;
  k.IN = c->IN;
  k.H = c->H;
  int64_t o = 0;
  for (int l = 0; l < c->L; ++l) {
    k.pk_off[l] = o;
    o += (int64_t)c->H * (l == 0 ? c->IN : c->H);
    k.w_off[l] = c->w_off[l];
    k.b_off[l] = c->b_off[l];
  }
  k.n_w = o;
  o = 0;
  for (int l = 0; l < c->L; ++l) {
    k.pkT_off[l] = o;
    if (l >= 1) o += (int64_t)c->H * c->H;
  }
  k.n_wt = o;
  k.wo_off = c->wo_off;
  return k;
}

inline size_t esize(int prec) { return prec == DINR_BF16 ? 2 : 4; }
