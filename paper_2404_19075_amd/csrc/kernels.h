// kernels.h -- argument blocks and launchers of the libdinr kernels
// (internal to the library; the public interface is include/dinr.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dinr_dev.h"

namespace dinr {

constexpr int MAX_LAYERS = 10;
// FWD: forward + ray-sum.  BWD: recomputed forward + adjoint from a given
// upstream gradient.  FUSED: forward, in-tile ray-sum, loss terms and the
// adjoint in one pass (tiles must hold whole rays).
// QUERY: points of queued requests (slices or reprojection rays) listed in a
// tile table; outputs mu0 M per point or ray-sums per ray.
// GROUP: the one-pass step for projections of several tiles (D x D rays of n
// samples, n a multiple of the tile): per group of tiles holding one
// projection, the forward of every tile, the projection's residual, then the
// adjoint of every tile (Swish networks, linear output).
enum { MODE_FWD = 0, MODE_BWD = 1, MODE_FUSED = 2, MODE_QUERY = 3, MODE_GROUP = 4 };

// One admitted query (device copy).  kind 0: n x n slice of mu0 M at height
// zn and time tn (normalised), pixel (i, j) at normalised (x, y) =
// (-1 + (2j+1)/n, -1 + (2i+1)/n).  kind 1: reprojection on an n x n detector
// covering the scanner's detector extent, view angle (cth, sth), time tn,
// `samples` equi-spaced samples per ray (a divisor of the tile size).
struct QueryDesc {
  int kind, n, samples, pad;
  float zn, tn, cth, sth;
  float* out;
};

struct QueryTile {
  int slot;  // descriptor index
  int tile;  // tile index within the query
};

struct GeomDev {
  int kind, rows, cols, n_views, fov_kind;
  int samp_mode, samp_n, samp_min, samp_max;
  float samp_h;
  int sub;  // D: D x D rays per projection
  float sod, sdd, pitch_u, pitch_v, off_u, off_v;
  float fov[6];
  float sc[3], oc[3];  // x_norm = x * sc + oc per axis (x, y, z)
  float mu0;
  const float* cth;    // [n_views] cos(theta_m)
  const float* sth;    // [n_views] sin(theta_m)
  const float* tnorm;  // [n_views] normalised time of view m
};

struct PackArgs {
  int L, IN, H;
  int64_t n_w, n_wt;                // packed elements, forward / transposed
  int64_t pk_off[MAX_LAYERS];       // element offset of layer l in the forward pack
  int64_t pkT_off[MAX_LAYERS];      // element offset of layer l (l >= 1) in the transposed pack
  int64_t w_off[MAX_LAYERS];        // offset of W_l in the flat parameters
  int64_t b_off[MAX_LAYERS];        // offset of b_l in the flat parameters
  int64_t wo_off;                   // offset of w_o
};

struct MlpArgs {
  const RayRec* rays;
  const int64_t* off;        // [R+1] point offsets
  const int32_t* tile_ray0;  // [n_tiles+1]
  int64_t R;
  const float4* Bmat;        // [C] GRFF rows (t, z, y, x)
  const float* params;       // flat FP32 parameters (for b_o)
  int64_t bo_off;
  const void* Wpk;
  const void* WTpk;
  const float* bias;         // [L][H]
  const float* wo_perm;      // [2][H/2] w_o in register-slot order
  int64_t wpk_off[MAX_LAYERS];
  int64_t wtpk_off[MAX_LAYERS];
  int64_t wpk_bytes, wtpk_bytes;  // sizes of the packed weight arrays
  int L, out_act;
  int act;                          // hidden activation: 0 ReLU, 1 Swish
  int jitter;                       // 1: stratified random sample positions
  uint32_t key0, key1;              // their generator's key (seed, epoch)
  int64_t tile_begin, tile_end;
  // group mode: tiles per group (one projection), tiles per ray, rays per
  // projection, projections
  int group_tiles, tiles_per_ray, d2;
  int64_t n_proj;
  // forward outputs
  float* part;               // [2 n_tiles] partial ray-sums
  float* proj;               // [R]
  // adjoint inputs/outputs
  const float* gup;          // [R] dL/dpbar
  void* stash;
  int64_t h_base[MAX_LAYERS];  // chunk (16 B) offsets of h_l blocks
  int64_t d_base[MAX_LAYERS];  // chunk offsets of delta_l blocks
  // chunk offsets of the Swish derivatives of h_l: the last layer's per point
  // (its weight gradient reads them); the other layers' in a ring of
  // ring_blocks 32-point blocks per workgroup, rewritten by every tile (group)
  // the workgroup takes, since only that tile's adjoint reads them
  int64_t a_base[MAX_LAYERS];
  int64_t ring_blocks;
  // delta_L is not stashed (L >= 2): its weight gradient rebuilds it from dL/dz_o
  // of every point (dob_base: 32 floats per 32-point block) and the last
  // layer's ReLU mask words (m_base: one 16-byte chunk per lane and block) or
  // its stashed Swish derivatives
  int64_t dob_base, m_base;
  float* opart;              // [grid][H+1] output-layer gradient partials
  // fused mode
  const float* meas;         // [R] measured projections
  double* lpart;             // [grid] partial sums of squared residuals
  // query mode
  const QueryDesc* qdesc;
  const QueryTile* qtiles;
  int64_t n_qtiles;
  GeomDev geom;
};

struct WgArgs {
  const int64_t* off;
  int64_t R;
  int tile;
  int64_t chunk_p0, chunk_p1;  // point range of this stash chunk
  int64_t kb;                  // 32-point blocks per split
  const void* stash;
  int64_t d_base, h_base;      // chunk offsets of this layer's delta / h blocks
  int coords;                  // h blocks hold point coordinates (layer 1): the
                               // encoding is re-derived with Bmat
  const float4* Bmat;          // [FI/2] GRFF rows (t, z, y, x)
  // the last layer (L >= 2): delta rebuilt as (w_o dL/dz_o) times the ReLU
  // mask (dmode 1) or times the stashed Swish derivative (dmode 2, m_base =
  // the layer's a_base); dmode 0: delta blocks at d_base
  int dmode;
  int64_t dob_base, m_base;
  const float* wo;             // [H] w_o in unit order
  float* wpart;                // [splits][nh]
  int64_t split_base, nh;
  int64_t w_off, b_off;
  int layer;
};

// One launch per stash chunk, in chunk order: the chunk's split partials are
// added to a running compensated sum (state: sums then compensations, nh
// floats each), so the result is that of one pass over every split in order.
struct RedArgs {
  const int64_t* off;
  int64_t R;
  int tile;
  int64_t chunk, chunk_points, kb;
  int first, last;             // first chunk: the sums start at zero; last:
                               // grad, the output-layer sums and grad^2 blocks
  const float* wpart;          // [splits of this chunk][nh]
  float* state;                // [2][nh]
  int64_t nh;
  const float* opart;
  int64_t n_opart, no;
  int64_t np;
  float* grad;
  double* gn_part;
};

// R projections -> R D^2 ray records; n_out (nullable) is per projection
hipError_t launch_bundle(const float* ray_proj, int64_t R, int D2, float* proj, hipStream_t st);
hipError_t launch_expand(const float* g_proj, int64_t R, int D2, float* g_ray, hipStream_t st);
// scan_ws: int64 [scan_blocks(R D^2)] of scratch for the offset scan
int64_t scan_blocks(int64_t n_rec);
// pad_n > 0: every ray record gets pad_n points (see k_rays)
hipError_t launch_rays(const GeomDev& g, const int64_t* idx, int64_t R, RayRec* rays, int32_t* nray,
                       int32_t* n_out, int64_t* off, int tile, int64_t n_tiles_max, int32_t* tr0,
                       int64_t* scan_ws, hipStream_t st, int pad_n = 0);
hipError_t launch_pack(int prec, const PackArgs& a, const float* P, void* Wpk, void* WTpk,
                       float* bias, float* wo, hipStream_t st);
hipError_t launch_mlp(int prec, int in, int h, int mode, const MlpArgs& a, int grid,
                      hipStream_t st);
hipError_t launch_query(int prec, int in, int h, const MlpArgs& a, int grid, hipStream_t st);
// one k_mlp instance (defined in mlp.h, instantiated in mlp_inst.hip)
template <int PREC, int IN, int H, int MODE, int ACT>
hipError_t mlp_launch(const MlpArgs& a, int grid, hipStream_t st);
hipError_t launch_fixup(const RayRec* rays, const int64_t* off, int64_t R, int tile,
                        const float* part, float* proj, hipStream_t st);
// lsum: double [LOSS_SCRATCH] of scratch for the per-workgroup partial sums
constexpr int LOSS_SCRATCH = 256;
hipError_t launch_loss(const float* proj, const float* meas, int64_t R, float* g, double* lsum,
                       double* loss, hipStream_t st);
// loss = (lpart sums + the terms of rays without samples) / n_div
hipError_t launch_loss_fused(const RayRec* rays, const float* meas, int64_t R, const double* lpart,
                             int64_t n_lpart, float* proj, double* lsum, double* loss,
                             int64_t n_div, hipStream_t st);
hipError_t launch_wgrad(int prec, int fi, int h, const WgArgs& a, int grid, hipStream_t st);
hipError_t launch_reduce(const RedArgs& a, double* gnorm_ws, double* gnorm_out, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2, const double* loss,
                       const double* gnorm, int32_t* status, hipStream_t st);

}  // namespace dinr
