// dinr_api.hip -- the C ABI of include/dinr.h: context, validation, the
// workspace arena and the launch sequences of forward projection, adjoint and
// training step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "ctx.h"

namespace {

struct Arena {
  char* base;
  size_t cap, used = 0;
  bool ok = true;
  template <class T>
  T* take(size_t n) {
    size_t off = (used + 255) & ~(size_t)255;
    size_t bytes = n * sizeof(T);
    if (off + bytes > cap) {
      ok = false;
      return nullptr;
    }
    used = off + bytes;
    return (T*)(base + off);
  }
};

// Everything one call needs, carved from the arena.
struct Plan {
  // R: ray records (Rp projections x D^2 rays each)
  int64_t R = 0, Rp = 0, D2 = 1, n_tiles_max = 0, points_max = 0;
  RayRec* rays = nullptr;
  int32_t* nray = nullptr;
  int64_t* off = nullptr;
  int32_t* tr0 = nullptr;
  int64_t* scan_ws = nullptr;  // block sums of the offset scan
  double* lsum = nullptr;      // per-workgroup partial sums of the loss
  float* part = nullptr;
  float* gup = nullptr;
  float* proj = nullptr;
  float* ray_proj = nullptr;  // D > 1: weighted sums of the single rays
  float* gproj = nullptr;     // D > 1: upstream gradient of the projections
  void* Wpk = nullptr;
  void* WTpk = nullptr;
  float* bias = nullptr;
  float* wo = nullptr;
  PackArgs pk{};
  // adjoint
  void* stash = nullptr;
  int64_t chunk_points = 0, n_chunks = 0, kb = 0, splits_per_chunk = 0;
  int64_t h_base[MAX_LAYERS], d_base[MAX_LAYERS], a_base[MAX_LAYERS];
  int64_t dob_base = 0, m_base = 0, ring_blocks = 0;
  float* wpart = nullptr;
  float* wstate = nullptr;  // running sums of the split partials over chunks
  float* opart = nullptr;
  double* lpart = nullptr;
  double* gn_part = nullptr;
  int grid_mlp = 0;
};

bool shape_supported(int in, int h) { return (in == 128 && h == 64) || (in == 256 && h == 256); }

}  // namespace

// ------------------------------------------------- static device scratch
//
// Scratch of dinr_forward_project_noalloc: ray records, offsets, tile map,
// tile partials and packed weights of one call, in a fixed array of the code
// object instead of the context's workspace.  Each device holds its own copy
// from the library's load until the process ends.  In host code `scratch`
// only names the symbol: its device address comes from hipGetSymbolAddress,
// looked up once per device by dinr_create with that device current.
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) char scratch[STATIC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[MAX_DEVICES] = {};
hipError_t g_scratch_err[MAX_DEVICES] = {};
bool g_scratch_done[MAX_DEVICES] = {};

// Device address of `scratch` on `dev` (the current device), resolved on the
// first call for that device; nullptr (and the HIP error in *err) if the
// lookup failed.
char* scratch_address(int dev, hipError_t* err) {
  if (dev < 0 || dev >= MAX_DEVICES) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      (void)hipGetLastError();  // keep the failure out of later calls' status
      ptr = nullptr;
    }
    g_scratch_ptr[dev] = (char*)ptr;
    g_scratch_err[dev] = e;
    g_scratch_done[dev] = true;
  }
  *err = g_scratch_err[dev];
  return g_scratch_ptr[dev];
}
}  // namespace

// Bytes at the start of the context's arena holding its status word and FP64
// scalars (loss, gradient norm); every call's plan is carved after them.
constexpr size_t ARENA_HEAD = 512;

// Carves the buffers of one call out of `A` (the context's arena after its
// head, or the library's static scratch).
static int plan_call(dinr_ctx* c, int64_t R, bool adjoint, Plan* p, Arena A) {
  p->Rp = R;
  p->D2 = (int64_t)c->gd.sub * c->gd.sub;
  p->R = R * p->D2;
  R = p->R;
  if (R > (int64_t)INT32_MAX - 1)
    return fail(c, DINR_EINVAL, "R D^2 = %lld rays exceeds 2^31 - 2", (long long)R);
  p->points_max = R * (int64_t)c->nmax;
  p->n_tiles_max = (p->points_max + c->tile - 1) / c->tile;
  p->rays = A.take<RayRec>(std::max<int64_t>(R, 1));
  p->nray = A.take<int32_t>(std::max<int64_t>(R, 1));
  p->off = A.take<int64_t>(R + 1);
  p->tr0 = A.take<int32_t>(p->n_tiles_max + 1);
  p->scan_ws = A.take<int64_t>(std::max<int64_t>(scan_blocks(R), 1));
  p->lsum = A.take<double>(LOSS_SCRATCH);
  p->part = A.take<float>(2 * std::max<int64_t>(p->n_tiles_max, 1));
  p->gup = A.take<float>(std::max<int64_t>(R, 1));
  p->proj = A.take<float>(std::max<int64_t>(p->Rp, 1));
  if (p->D2 > 1) {
    p->ray_proj = A.take<float>(R);
    p->gproj = A.take<float>(p->Rp);
  }
  // packed weights
  p->pk = pack_layout(c);
  const PackArgs& k = p->pk;
  p->Wpk = A.take<char>(k.n_w * esize(c->prec));
  p->WTpk = A.take<char>(std::max<int64_t>(k.n_wt, 1) * esize(c->prec));
  p->bias = A.take<float>((size_t)c->L * c->H);
  p->wo = A.take<float>(c->H);
  p->grid_mlp = c->n_cu;
  if (!A.ok) return fail(c, DINR_ENOMEM, "workspace budget too small for R=%lld", (long long)R);
  if (!adjoint) return DINR_OK;

  // adjoint: split partials for one stash chunk, output-layer partials per
  // chunk, then as large a stash chunk as the remaining budget allows.  A
  // weight-gradient workgroup sums a split of 4,096 to 65,536 points, chosen
  // below once the chunk size is known (the stash chunks are multiples of
  // 16,384 points)
  const int64_t ks_min = 4096, ks_max = 65536, k_chunk = 16384;
  // stash bytes per point: layer 1's input as the point's 4 coordinates (16
  // bytes), h_1 .. h_{L-1} and delta_1 .. delta_{L-1}; delta_L (L >= 2) as
  // dL/dz_o (4 bytes) and, ReLU, the last layer's mask bits (32 bytes per
  // point at H = 256, one 16-byte chunk per lane and 32-point block); Swish: the
  // last layer's activation derivatives as well.  The Swish derivatives of the
  // other layers are read only by the adjoint of the same tile: they live in a
  // ring per workgroup of the persistent kernel, one tile deep (the group of
  // tiles of one projection in the grouped one-pass step).
  const int64_t hb = (int64_t)c->H * esize(c->prec);
  const bool compact = c->L >= 2;
  const bool swish = c->mlp.act == DINR_SWISH;
  int64_t per_point = 16;
  for (int l = 1; l < c->L; ++l) per_point += hb;
  per_point += (int64_t)(compact ? c->L - 1 : c->L) * hb;
  if (compact) per_point += 4 + (swish ? 0 : 32);
  if (swish) per_point += hb;
  const int vpc2 = (c->prec == DINR_BF16 ? 8 : 4) * 2;  // features per 16-byte lane pair
  const int64_t layer_chunks = (int64_t)(c->H / vpc2) * 64;  // per 32-point block and layer
  const int64_t group = c->samp.mode == 0 ? p->D2 * c->samp.n / c->tile : 0;
  p->ring_blocks = (group >= 2 && group <= 64 ? group : 1) * (c->tile / 32);
  const int64_t ring_chunks = swish ? (int64_t)(c->L - 1) * p->grid_mlp * p->ring_blocks *
                                          layer_chunks : 0;
  const int64_t quantum = std::max<int64_t>(k_chunk, c->tile);  // both powers of two
  const int64_t pts_pad = std::max<int64_t>((p->points_max + quantum - 1) / quantum * quantum, quantum);
  // partials of one chunk: up to 2 n_cu splits (no more than one per 16,384
  // points of the batch), or one per 65,536 points of the batch when that is
  // more; the split size below keeps every chunk within this
  const int64_t max_splits = std::max<int64_t>(std::min<int64_t>(2 * c->n_cu, pts_pad / k_chunk),
                                               (pts_pad + ks_max - 1) / ks_max);
  p->wpart = A.take<float>((size_t)max_splits * c->nh);
  p->wstate = A.take<float>((size_t)2 * c->nh);
  p->gn_part = A.take<double>((size_t)((c->np + 255) / 256));
  if (!A.ok) return fail(c, DINR_ENOMEM, "workspace budget too small for the gradient partials");
  // try the whole batch in one chunk, then halve
  int64_t chunk = pts_pad;
  const size_t used0 = A.used;
  for (;;) {
    A.used = used0;
    A.ok = true;
    const int64_t n_chunks = (pts_pad + chunk - 1) / chunk;
    p->opart = A.take<float>((size_t)n_chunks * p->grid_mlp * (c->H + 1));
    p->lpart = A.take<double>((size_t)n_chunks * p->grid_mlp);
    p->stash = A.take<char>((size_t)ring_chunks * 16 + (size_t)chunk * per_point);
    if (A.ok) {
      p->chunk_points = chunk;
      p->n_chunks = n_chunks;
      break;
    }
    if (chunk <= quantum)
      return fail(c, DINR_ENOMEM, "workspace budget too small for a stash of %lld points",
                  (long long)chunk);
    chunk = std::max<int64_t>(quantum, (chunk / 2 + quantum - 1) / quantum * quantum);
  }
  // the largest split (a power of two, 4,096 to 65,536 points) that still
  // gives each compute unit a split of the chunk, as long as the chunk's
  // partials fit: fewer partials to write and to combine, and a full grid for
  // small chunks.  The chunk's last split may be partial; at 65,536 points a
  // chunk has at most pts_pad / 65,536 splits, so the loop ends within bounds
  int64_t ks = ks_min;
  while (ks < ks_max && (p->chunk_points / (2 * ks) >= c->n_cu ||
                         (p->chunk_points + ks - 1) / ks > max_splits))
    ks *= 2;
  p->kb = ks / 32;
  p->splits_per_chunk = (p->chunk_points + ks - 1) / ks;
  if (p->splits_per_chunk > max_splits) return fail(c, DINR_EINVAL, "split plan");
  // the Swish derivative ring (layers 1 .. L-1), then the stash region of each
  // layer: h blocks then delta blocks, in 16-byte chunks
  for (int l = 0; l + 1 < c->L; ++l)
    p->a_base[l] = swish ? (int64_t)l * p->grid_mlp * p->ring_blocks * layer_chunks : 0;
  int64_t base = ring_chunks;
  const int64_t blocks = p->chunk_points / 32;
  for (int l = 0; l < c->L; ++l) {
    p->h_base[l] = base;
    // layer 1: one 16-byte chunk of coordinates per point
    base += l == 0 ? p->chunk_points : blocks * layer_chunks;
    p->d_base[l] = base;
    if (!(compact && l == c->L - 1)) base += blocks * layer_chunks;
  }
  p->a_base[c->L - 1] = base;
  if (swish) base += blocks * layer_chunks;
  // delta_L's substitutes: 32 floats (8 chunks) of dL/dz_o and, ReLU, 64 mask
  // chunks per block
  p->dob_base = base;
  if (compact) base += blocks * 8;
  p->m_base = base;
  if (compact && c->mlp.act != DINR_SWISH) base += blocks * 64;
  return DINR_OK;
}

static int plan_call(dinr_ctx* c, int64_t R, bool adjoint, Plan* p) {
  return plan_call(c, R, adjoint, p, Arena{c->arena + ARENA_HEAD, c->arena_size - ARENA_HEAD});
}

static MlpArgs mlp_args(dinr_ctx* c, const Plan& p, const float* params) {
  MlpArgs a{};
  a.rays = p.rays;
  a.off = p.off;
  a.tile_ray0 = p.tr0;
  a.R = p.R;
  a.Bmat = c->d_B;
  a.params = params;
  a.bo_off = c->bo_off;
  a.Wpk = p.Wpk;
  a.WTpk = p.WTpk;
  a.bias = p.bias;
  a.wo_perm = p.wo;
  for (int l = 0; l < c->L; ++l) {
    a.wpk_off[l] = p.pk.pk_off[l];
    a.wtpk_off[l] = p.pk.pkT_off[l];
  }
  a.wpk_bytes = p.pk.n_w * (int64_t)esize(c->prec);
  a.wtpk_bytes = p.pk.n_wt * (int64_t)esize(c->prec);
  a.L = c->L;
  a.out_act = c->mlp.out_act;
  a.act = c->mlp.act == DINR_SWISH ? 1 : 0;
  a.jitter = c->samp.jitter != 0;
  a.key0 = c->samp.seed;
  a.key1 = c->epoch;
  a.tile_begin = 0;
  a.tile_end = p.n_tiles_max;
  a.part = p.part;
  a.proj = nullptr;
  return a;
}

static int enqueue_forward(dinr_ctx* c, const Plan& p, const float* params,
                           const int64_t* idx, float* proj, int32_t* n_out, hipStream_t st) {
  {
    ProfScope ps(c, DINR_PROF_RAYS, st);
    HIPCHK(c, launch_rays(c->gd, idx, p.Rp, p.rays, p.nray, n_out, p.off, c->tile, p.n_tiles_max,
                          p.tr0, p.scan_ws, st));
  }
  HIPCHK(c, launch_pack(c->prec == DINR_BF16 ? PREC_BF16 : PREC_F32, p.pk, params, p.Wpk, p.WTpk,
                        p.bias, p.wo, st));
  MlpArgs a = mlp_args(c, p, params);
  // the kernel writes one sum per ray record: with D > 1 those are the single
  // rays, summed into the projections below
  float* ray_out = p.D2 > 1 ? p.ray_proj : proj;
  a.proj = ray_out;
  {
    ProfScope ps(c, DINR_PROF_MLP_FWD, st);
    HIPCHK(c, launch_mlp(c->prec == DINR_BF16 ? PREC_BF16 : PREC_F32, c->IN, c->H, MODE_FWD, a,
                         p.grid_mlp, st));
  }
  HIPCHK(c, launch_fixup(p.rays, p.off, p.R, c->tile, p.part, ray_out, st));
  if (p.D2 > 1) {
    ProfScope ps(c, DINR_PROF_LOSS, st);
    HIPCHK(c, launch_bundle(p.ray_proj, p.Rp, (int)p.D2, proj, st));
  }
  return DINR_OK;
}

// Adjoint (rays, offsets and packed weights already in place).  mode
// MODE_BWD: upstream gradient given in gup, forward recomputed per tile.
// MODE_FUSED: forward, ray-sums, residuals against meas and the adjoint in
// one pass; proj receives the predictions and lpart the residual sums.
// MODE_GROUP: as MODE_FUSED for projections of group_tiles tiles each (the
// rays padded to n points, n a multiple of the tile).
static int enqueue_adjoint(dinr_ctx* c, const Plan& p, const float* params, const float* gup,
                           float* grad, double* gnorm_out, hipStream_t st, int mode = MODE_BWD,
                           const float* meas = nullptr, float* proj = nullptr,
                           int group_tiles = 1) {
  const int prec = c->prec == DINR_BF16 ? PREC_BF16 : PREC_F32;
  const int64_t tiles_per_chunk = p.chunk_points / c->tile;
  for (int64_t ch = 0; ch < p.n_chunks; ++ch) {
    MlpArgs a = mlp_args(c, p, params);
    a.tile_begin = ch * tiles_per_chunk;
    a.tile_end = std::min<int64_t>((ch + 1) * tiles_per_chunk, p.n_tiles_max);
    a.group_tiles = group_tiles;
    a.tiles_per_ray = group_tiles / (int)p.D2;
    a.d2 = (int)p.D2;
    a.n_proj = p.Rp;
    a.gup = gup;
    a.meas = meas;
    a.proj = proj;
    a.lpart = p.lpart + ch * (int64_t)p.grid_mlp;
    a.stash = p.stash;
    for (int l = 0; l < c->L; ++l) {
      a.h_base[l] = p.h_base[l];
      a.d_base[l] = p.d_base[l];
      a.a_base[l] = p.a_base[l];
    }
    a.ring_blocks = p.ring_blocks;
    a.dob_base = p.dob_base;
    a.m_base = p.m_base;
    a.opart = p.opart + ch * (int64_t)p.grid_mlp * (c->H + 1);
    {
      ProfScope ps(c, mode == MODE_BWD ? DINR_PROF_MLP_BWD : DINR_PROF_MLP_FUSED, st);
      HIPCHK(c, launch_mlp(prec, c->IN, c->H, mode, a, p.grid_mlp, st));
    }
    for (int l = 0; l < c->L; ++l) {
      WgArgs w{};
      w.off = p.off;
      w.R = p.R;
      w.tile = c->tile;
      w.chunk_p0 = ch * p.chunk_points;
      w.chunk_p1 = (ch + 1) * p.chunk_points;
      w.kb = p.kb;
      w.stash = p.stash;
      w.d_base = p.d_base[l];
      w.h_base = p.h_base[l];
      w.coords = l == 0;
      w.Bmat = c->d_B;
      // the last layer's delta is rebuilt (L >= 2)
      w.dmode = (c->L >= 2 && l == c->L - 1) ? (c->mlp.act == DINR_SWISH ? 2 : 1) : 0;
      w.dob_base = p.dob_base;
      w.m_base = c->mlp.act == DINR_SWISH ? p.a_base[l] : p.m_base;
      w.wo = params + c->wo_off;
      w.wpart = p.wpart;
      w.split_base = 0;  // one chunk's partials, combined after its launches
      w.nh = c->nh;
      w.w_off = c->w_off[l];
      w.b_off = c->b_off[l];
      w.layer = l;
      ProfScope ps(c, DINR_PROF_WGRAD, st);
      HIPCHK(c, launch_wgrad(prec, l == 0 ? c->IN : c->H, c->H, w, (int)p.splits_per_chunk, st));
    }
    RedArgs r{};
    r.off = p.off;
    r.R = p.R;
    r.tile = c->tile;
    r.chunk = ch;
    r.chunk_points = p.chunk_points;
    r.kb = p.kb;
    r.first = ch == 0;
    r.last = ch + 1 == p.n_chunks;
    r.wpart = p.wpart;
    r.state = p.wstate;
    r.nh = c->nh;
    r.opart = p.opart;
    r.n_opart = p.n_chunks * p.grid_mlp;
    r.no = c->H + 1;
    r.np = c->np;
    r.grad = grad;
    r.gn_part = p.gn_part;
    if (r.last && (mode == MODE_FUSED || mode == MODE_GROUP)) {
      // the grouped step computed every projection's loss term in the kernel
      ProfScope ps(c, DINR_PROF_LOSS, st);
      HIPCHK(c, launch_loss_fused(p.rays, meas, mode == MODE_GROUP ? 0 : p.R, p.lpart,
                                  p.n_chunks * p.grid_mlp, proj, p.lsum, c->d_scal, p.Rp, st));
    }
    ProfScope ps(c, DINR_PROF_REDUCE, st);
    HIPCHK(c, launch_reduce(r, c->d_scal + 1, gnorm_out, st));
  }
  return DINR_OK;
}

extern "C" {

int dinr_create(const dinr_geometry* g, const dinr_mlp* m, const dinr_sampling* s,
                const float* B_host, size_t budget, dinr_ctx** out) {
  if (!out) return DINR_EINVAL;
  *out = nullptr;
  if (!g || !m || !s || !B_host) return DINR_EINVAL;
  dinr_ctx* c = new (std::nothrow) dinr_ctx();
  if (!c) return DINR_ENOMEM;
  auto bad = [&](const char* msg) {
    fail(c, DINR_EINVAL, "%s", msg);
    return DINR_EINVAL;
  };
  int rc = DINR_OK;
  do {
    if (g->kind != DINR_PARALLEL && g->kind != DINR_CONE) { rc = bad("geometry kind"); break; }
    if (g->rows <= 0 || g->cols <= 0 || g->n_views <= 0) { rc = bad("detector shape"); break; }
    if (!g->theta || !g->time) { rc = bad("theta/time tables"); break; }
    if (g->kind == DINR_CONE && !(g->sdd > 0 && g->sod > 0 && g->sdd > g->sod)) {
      rc = bad("cone geometry needs 0 < sod < sdd");
      break;
    }
    if (!(g->pitch_u > 0 && g->pitch_v > 0)) { rc = bad("pixel pitch"); break; }
    if (g->fov_kind == DINR_FOV_BOX) {
      if (!(g->fov[1] > g->fov[0] && g->fov[3] > g->fov[2] && g->fov[5] > g->fov[4])) {
        rc = bad("box FOV bounds");
        break;
      }
    } else if (g->fov_kind == DINR_FOV_CYLINDER) {
      if (!(g->fov[0] > 0 && g->fov[2] > g->fov[1])) { rc = bad("cylinder FOV"); break; }
    } else {
      rc = bad("fov_kind");
      break;
    }
    if (!(g->t1 > g->t0)) { rc = bad("time range"); break; }
    const int IN = 2 * m->n_freq, H = m->width;
    if (!shape_supported(IN, H)) { rc = bad("unsupported (2C, H): supported (128,64), (256,256)"); break; }
    if (m->depth < 1 || m->depth > MAX_LAYERS) { rc = bad("depth must be in [1, 10]"); break; }
    if (m->act != DINR_RELU && m->act != DINR_SWISH) { rc = bad("act"); break; }
    if (m->out_act != DINR_OUT_IDENTITY && m->out_act != DINR_OUT_SOFTPLUS) { rc = bad("out_act"); break; }
    if (m->precision != DINR_FP32 && m->precision != DINR_BF16) { rc = bad("precision"); break; }
    if (!std::isfinite(m->mu0)) { rc = bad("mu0"); break; }
    if (s->mode == 0) {
      if (s->n < 1 || s->n > (1 << 20)) { rc = bad("samples per ray"); break; }
    } else if (s->mode == 1) {
      if (!(s->h > 0) || s->n_min < 1 || s->n_max < s->n_min || s->n_max > (1 << 20)) {
        rc = bad("step sampling");
        break;
      }
    } else {
      rc = bad("sampling mode");
      break;
    }
    if (s->sub < 0 || s->sub > 8) { rc = bad("rays per projection: D must be in [1, 8]"); break; }
    if (s->jitter != 0 && s->jitter != 1) { rc = bad("jitter must be 0 or 1"); break; }
    for (int k = 0; k < 4 * m->n_freq; ++k)
      if (!std::isfinite(B_host[k])) { rc = bad("B has a non-finite entry"); break; }
    if (rc) break;
    for (int v = 0; v < g->n_views; ++v)
      if (!std::isfinite(g->theta[v]) || !std::isfinite(g->time[v])) { rc = bad("theta/time"); break; }
    if (rc) break;
    if (budget < ((size_t)8 << 20)) {
      rc = fail(c, DINR_ENOMEM, "workspace budget below 8 MiB");
      break;
    }
  } while (0);
  if (rc) {
    // keep the message reachable: a context that failed creation is returned
    // only through the error code, so print nothing and free it
    delete c;
    return rc;
  }
  c->geom = *g;
  c->geom.theta = nullptr;
  c->geom.time = nullptr;
  c->mlp = *m;
  c->samp = *s;
  c->IN = 2 * m->n_freq;
  c->H = m->width;
  c->L = m->depth;
  c->prec = m->precision;
  c->tile = m->precision == DINR_BF16 ? Prec<PREC_BF16>::WAVES * Prec<PREC_BF16>::NB * 32
                                      : Prec<PREC_F32>::WAVES * Prec<PREC_F32>::NB * 32;
  c->nmax = s->mode == 0 ? s->n : s->n_max;
  int64_t o = 0;
  for (int l = 0; l < c->L; ++l) {
    const int fin = l == 0 ? c->IN : c->H;
    c->w_off.push_back(o);
    o += (int64_t)c->H * fin;
    c->b_off.push_back(o);
    o += c->H;
  }
  c->nh = o;
  c->wo_off = o;
  c->bo_off = o + c->H;
  c->np = o + c->H + 1;

  hipError_t e = hipGetDevice(&c->device);
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, c->device);
  if (e != hipSuccess) {
    delete c;
    return DINR_EHIP;
  }
  c->n_cu = prop.multiProcessorCount;
  {
    // resolve the static scratch of this device now, with it current
    hipError_t se = hipSuccess;
    (void)scratch_address(c->device, &se);
  }
  const int nv = g->n_views;
  std::vector<float> cth(nv), sth(nv), tn(nv);
  for (int v = 0; v < nv; ++v) {
    cth[v] = (float)std::cos(g->theta[v]);
    sth[v] = (float)std::sin(g->theta[v]);
    tn[v] = (float)(2.0 * (g->time[v] - g->t0) / (g->t1 - g->t0) - 1.0);
  }
  std::vector<float> Bv(4 * m->n_freq);
  std::memcpy(Bv.data(), B_host, sizeof(float) * Bv.size());
  if (hipMalloc(&c->d_cth, nv * sizeof(float)) != hipSuccess ||
      hipMalloc(&c->d_sth, nv * sizeof(float)) != hipSuccess ||
      hipMalloc(&c->d_tn, nv * sizeof(float)) != hipSuccess ||
      hipMalloc(&c->d_B, Bv.size() * sizeof(float)) != hipSuccess ||
      hipMalloc(&c->arena, budget) != hipSuccess) {
    dinr_destroy(c);
    return DINR_ENOMEM;
  }
  c->arena_size = budget;
  c->d_status = (int32_t*)c->arena;
  c->d_scal = (double*)(c->arena + 256);
  if (hipMemcpy(c->d_cth, cth.data(), nv * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_sth, sth.data(), nv * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_tn, tn.data(), nv * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->d_B, Bv.data(), Bv.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
    dinr_destroy(c);
    return DINR_EHIP;
  }
  GeomDev& d = c->gd;
  d.kind = g->kind;
  d.rows = g->rows;
  d.cols = g->cols;
  d.n_views = g->n_views;
  d.fov_kind = g->fov_kind;
  d.samp_mode = s->mode;
  d.samp_n = s->n;
  d.samp_min = s->n_min;
  d.samp_max = s->n_max;
  d.samp_h = (float)s->h;
  d.sub = s->sub > 1 ? s->sub : 1;
  d.sod = (float)g->sod;
  d.sdd = (float)g->sdd;
  d.pitch_u = (float)g->pitch_u;
  d.pitch_v = (float)g->pitch_v;
  d.off_u = (float)g->off_u;
  d.off_v = (float)g->off_v;
  for (int k = 0; k < 6; ++k) d.fov[k] = (float)g->fov[k];
  double lo[3], hi[3];
  if (g->fov_kind == DINR_FOV_BOX) {
    for (int a = 0; a < 3; ++a) { lo[a] = g->fov[2 * a]; hi[a] = g->fov[2 * a + 1]; }
  } else {
    lo[0] = lo[1] = -g->fov[0];
    hi[0] = hi[1] = g->fov[0];
    lo[2] = g->fov[1];
    hi[2] = g->fov[2];
  }
  for (int a = 0; a < 3; ++a) {
    d.sc[a] = (float)(2.0 / (hi[a] - lo[a]));
    d.oc[a] = (float)(-2.0 * lo[a] / (hi[a] - lo[a]) - 1.0);
  }
  d.mu0 = (float)m->mu0;
  d.cth = c->d_cth;
  d.sth = c->d_sth;
  d.tnorm = c->d_tn;
  *out = c;
  return DINR_OK;
}

int dinr_destroy(dinr_ctx* c) {
  if (!c) return DINR_OK;
  for (int k = 0; k < DINR_PROF_KINDS; ++k)
    for (int j = 0; j < 2; ++j)
      for (auto& e : c->prof.ev[k][j]) hipEventDestroy(e);
  hipFree(c->d_cth);
  hipFree(c->d_sth);
  hipFree(c->d_tn);
  hipFree(c->d_B);
  hipFree(c->arena);
  delete c;
  return DINR_OK;
}

const char* dinr_last_error(const dinr_ctx* c) { return c ? c->err : "null context"; }

int dinr_set_sample_epoch(dinr_ctx* c, uint32_t epoch) {
  if (!c) return DINR_EINVAL;
  c->epoch = epoch;
  return DINR_OK;
}

int dinr_profile_enable(dinr_ctx* c, int enable) {
  if (!c) return DINR_EINVAL;
  auto& p = c->prof;
  if (enable && p.ev[0][0].empty()) {
    for (int k = 0; k < DINR_PROF_KINDS; ++k)
      for (int j = 0; j < 2; ++j) {
        p.ev[k][j].resize(4096);
        for (auto& e : p.ev[k][j]) HIPCHK(c, hipEventCreate(&e));
      }
  }
  p.on = enable != 0;
  for (int k = 0; k < DINR_PROF_KINDS; ++k) p.used[k] = 0;
  return DINR_OK;
}

int dinr_profile_read(dinr_ctx* c, int kind, double* total_ms, int64_t* launches) {
  if (!c || kind < 0 || kind >= DINR_PROF_KINDS || !total_ms || !launches) return DINR_EINVAL;
  auto& p = c->prof;
  double t = 0.0;
  for (size_t i = 0; i < p.used[kind]; ++i) {
    HIPCHK(c, hipEventSynchronize(p.ev[kind][1][i]));
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, p.ev[kind][0][i], p.ev[kind][1][i]));
    t += ms;
  }
  *total_ms = t;
  *launches = (int64_t)p.used[kind];
  p.used[kind] = 0;
  return DINR_OK;
}

int64_t dinr_num_params(const dinr_ctx* c) { return c ? c->np : -1; }

int dinr_forward_project(dinr_ctx* c, const float* params, const int64_t* idx, int64_t R,
                         float* proj, int32_t* n_out, void* stream) {
  if (!c) return DINR_EINVAL;
  if (R < 0 || R > (int64_t)INT32_MAX - 1) return fail(c, DINR_EINVAL, "R out of range");
  if (R > 0 && (!params || !idx || !proj)) return fail(c, DINR_EINVAL, "null buffer");
  if (R == 0) return DINR_OK;
  hipStream_t st = (hipStream_t)stream;
  Plan p;
  int rc = plan_call(c, R, false, &p);
  if (rc) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  return enqueue_forward(c, p, params, idx, proj, n_out, st);
}

int dinr_forward_project_noalloc(dinr_ctx* c, const float* params, const int64_t* idx, int64_t R,
                                 float* proj, int32_t* n_out, void* stream) {
  if (!c) return DINR_EINVAL;
  if (R < 0 || R > (int64_t)INT32_MAX - 1) return fail(c, DINR_EINVAL, "R out of range");
  if (R > 0 && (!params || !idx || !proj)) return fail(c, DINR_EINVAL, "null buffer");
  if (R == 0) return DINR_OK;
  hipError_t se = hipSuccess;
  char* base = scratch_address(c->device, &se);
  if (!base)
    return fail(c, DINR_EHIP, "static scratch of device %d unavailable: %s", c->device,
                hipGetErrorString(se));
  Plan p;
  int rc = plan_call(c, R, false, &p, Arena{base, STATIC_SCRATCH_BYTES});
  if (rc)
    return fail(c, DINR_ENOMEM,
                "R=%lld needs more than the %zu-byte static scratch of the no-allocation "
                "forward projection", (long long)R, STATIC_SCRATCH_BYTES);
  HIPCHK(c, hipSetDevice(c->device));
  return enqueue_forward(c, p, params, idx, proj, n_out, (hipStream_t)stream);
}

int dinr_project_backward(dinr_ctx* c, const float* params, const int64_t* idx, int64_t R,
                          const float* dproj, float* grad, double* gnorm, void* stream) {
  if (!c) return DINR_EINVAL;
  if (R < 0 || R > (int64_t)INT32_MAX - 1) return fail(c, DINR_EINVAL, "R out of range");
  if (!params || !grad || (R > 0 && (!idx || !dproj))) return fail(c, DINR_EINVAL, "null buffer");
  hipStream_t st = (hipStream_t)stream;
  Plan p;
  int rc = plan_call(c, R, true, &p);
  if (rc) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  {
    ProfScope ps(c, DINR_PROF_RAYS, st);
    HIPCHK(c, launch_rays(c->gd, idx, R, p.rays, p.nray, nullptr, p.off, c->tile, p.n_tiles_max,
                          p.tr0, p.scan_ws, st));
  }
  HIPCHK(c, launch_pack(c->prec == DINR_BF16 ? PREC_BF16 : PREC_F32, p.pk, params, p.Wpk, p.WTpk,
                        p.bias, p.wo, st));
  if (p.D2 > 1) {
    HIPCHK(c, launch_expand(dproj, R, (int)p.D2, p.gup, st));
    dproj = p.gup;
  }
  return enqueue_adjoint(c, p, params, dproj, grad, gnorm, st);
}

int dinr_step(dinr_ctx* c, float* params, const int64_t* idx, int64_t R, const float* meas,
              float* proj_out, float* grad, double* loss, double* gnorm, const dinr_adam* adam,
              void* stream) {
  if (!c) return DINR_EINVAL;
  if (R < 1 || R > (int64_t)INT32_MAX - 1) return fail(c, DINR_EINVAL, "R out of range");
  if (!params || !idx || !meas || !grad) return fail(c, DINR_EINVAL, "null buffer");
  if (adam) {
    if (!adam->m_d || !adam->v_d) return fail(c, DINR_EINVAL, "Adam state buffers");
    if (adam->step < 1) return fail(c, DINR_EINVAL, "Adam step must be >= 1");
    if (!(adam->lr > 0) || !(adam->beta1 >= 0 && adam->beta1 < 1) ||
        !(adam->beta2 >= 0 && adam->beta2 < 1) || !(adam->eps > 0))
      return fail(c, DINR_EINVAL, "Adam hyper-parameters");
  }
  hipStream_t st = (hipStream_t)stream;
  Plan p;
  int rc = plan_call(c, R, true, &p);
  if (rc) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  float* proj = proj_out ? proj_out : p.proj;
  // one pass when every tile holds whole projections: fixed n dividing the
  // tile, one ray per projection
  const bool fused = !c->mlp.recompute && c->samp.mode == 0 && c->tile % c->samp.n == 0 &&
                     p.D2 == 1;
  // one pass over groups of tiles, each holding one projection, when its rays
  // have n samples, n a multiple of the tile (Swish network, linear output:
  // the adjoint reads the activation derivatives back from the stash), and
  // the stash chunks hold whole groups
  const int64_t group = c->samp.mode == 0 ? p.D2 * c->samp.n / c->tile : 0;
  const bool grouped = !fused && !c->mlp.recompute && c->samp.mode == 0 &&
                       c->samp.n % c->tile == 0 && c->mlp.act == DINR_SWISH &&
                       c->mlp.out_act == DINR_OUT_IDENTITY && c->L >= 2 && group >= 2 &&
                       group <= 64 && (p.chunk_points / c->tile) % group == 0;
  if (grouped) {
    {
      ProfScope ps(c, DINR_PROF_RAYS, st);
      HIPCHK(c, launch_rays(c->gd, idx, R, p.rays, p.nray, nullptr, p.off, c->tile,
                            p.n_tiles_max, p.tr0, p.scan_ws, st, c->samp.n));
    }
    HIPCHK(c, launch_pack(c->prec == DINR_BF16 ? PREC_BF16 : PREC_F32, p.pk, params, p.Wpk,
                          p.WTpk, p.bias, p.wo, st));
    rc = enqueue_adjoint(c, p, params, nullptr, grad, gnorm, st, MODE_GROUP, meas, proj,
                         (int)group);
    if (rc) return rc;
    if (loss)
      HIPCHK(c, hipMemcpyAsync(loss, c->d_scal, sizeof(double), hipMemcpyDeviceToDevice, st));
  } else if (fused) {
    {
      ProfScope ps(c, DINR_PROF_RAYS, st);
      HIPCHK(c, launch_rays(c->gd, idx, R, p.rays, p.nray, nullptr, p.off, c->tile,
                            p.n_tiles_max, p.tr0, p.scan_ws, st));
    }
    HIPCHK(c, launch_pack(c->prec == DINR_BF16 ? PREC_BF16 : PREC_F32, p.pk, params, p.Wpk,
                          p.WTpk, p.bias, p.wo, st));
    rc = enqueue_adjoint(c, p, params, nullptr, grad, gnorm, st, MODE_FUSED, meas, proj);
    if (rc) return rc;
    if (loss)
      HIPCHK(c, hipMemcpyAsync(loss, c->d_scal, sizeof(double), hipMemcpyDeviceToDevice, st));
  } else {
    rc = enqueue_forward(c, p, params, idx, proj, nullptr, st);
    if (rc) return rc;
    {
      ProfScope ps(c, DINR_PROF_LOSS, st);
      HIPCHK(c, launch_loss(proj, meas, R, p.D2 > 1 ? p.gproj : p.gup, p.lsum, c->d_scal, st));
      if (p.D2 > 1) HIPCHK(c, launch_expand(p.gproj, R, (int)p.D2, p.gup, st));
    }
    if (loss)
      HIPCHK(c, hipMemcpyAsync(loss, c->d_scal, sizeof(double), hipMemcpyDeviceToDevice, st));
    rc = enqueue_adjoint(c, p, params, p.gup, grad, gnorm, st);
    if (rc) return rc;
  }
  if (adam) {
    const float c1 = (float)(1.0 - std::pow((double)adam->beta1, (double)adam->step));
    const float c2 = (float)(1.0 - std::pow((double)adam->beta2, (double)adam->step));
    HIPCHK(c, launch_adam(params, grad, adam->m_d, adam->v_d, c->np, adam->lr, adam->beta1,
                          adam->beta2, adam->eps, c1, c2, c->d_scal, c->d_scal + 1, c->d_status,
                          st));
  }
  return DINR_OK;
}

int dinr_step_status(dinr_ctx* c, void* stream) {
  if (!c) return DINR_EINVAL;
  double sc[2] = {0.0, 0.0};
  HIPCHK(c, hipMemcpyAsync(sc, c->d_scal, 2 * sizeof(double), hipMemcpyDeviceToHost,
                           (hipStream_t)stream));
  HIPCHK(c, hipStreamSynchronize((hipStream_t)stream));
  if (!std::isfinite(sc[0]) || !std::isfinite(sc[1]))
    return fail(c, DINR_ENONFINITE, "loss or gradient norm not finite; Adam step skipped");
  return DINR_OK;
}

}  // extern "C"
