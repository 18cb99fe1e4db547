/*
 * dinr.h -- C ABI of libdinr, the gfx950 (MI355X) implementation of one DINR
 * training step over a sparse batch of detector rays, its forward projection
 * and adjoint, and queries of the trained field.
 *
 * Method: Mohan et al., "Distributed Stochastic Optimization of a Neural
 * Representation Network for Time-Space Tomography Reconstruction"
 * (arXiv 2404.19075).  Section and equation numbers below are that paper's.
 *
 * Conventions shared by every entry point
 *  - Pointers named *_d are device pointers (hipMalloc'd or torch-allocated
 *    on the context's device); pointers without the suffix are host pointers.
 *    The caller owns every buffer it passes; the library never frees them.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Calls only enqueue work on that stream; outputs are valid after the
 *    stream is synchronised.  Calls on one context must not overlap in time
 *    (the context's workspace is shared); use one context per stream.
 *  - Errors are negative return values; dinr_last_error() gives a message.
 *    Argument errors are detected before anything is enqueued, and then no
 *    output or parameter buffer is touched.  No exception crosses the ABI.
 *  - The context allocates one device workspace of `workspace_budget` bytes
 *    in dinr_create and nothing afterwards; a batch that cannot be processed
 *    within it (even in chunks) is rejected with DINR_ENOMEM.
 *  - Parameters gamma are one flat FP32 vector: for each hidden layer
 *    l = 1..L, W_l [H x fan_in] row-major (row = output unit) then b_l [H];
 *    then the output layer w_o [H] and b_o [1].  fan_in = 2C for l = 1 and
 *    H otherwise.  Gradients use the same layout.
 */
#ifndef DINR_H
#define DINR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DINR_OK = 0,
  DINR_EINVAL = -1,      /* bad argument, geometry or shape */
  DINR_ENOMEM = -2,      /* workspace budget too small, or allocation failed */
  DINR_EHIP = -3,        /* a HIP runtime call failed */
  DINR_ENONFINITE = -4,  /* loss or gradient norm is not finite; Adam skipped */
  DINR_EBUSY = -5,       /* serving: admission refused (budget or slots full) */
  DINR_EIO = -6          /* volume writer: the output file could not be written */
};

enum { DINR_PARALLEL = 0, DINR_CONE = 1 };
enum { DINR_FOV_BOX = 0, DINR_FOV_CYLINDER = 1 };
enum { DINR_RELU = 0, DINR_SWISH = 1 };
enum { DINR_OUT_IDENTITY = 0, DINR_OUT_SOFTPLUS = 1 };
enum { DINR_FP32 = 0, DINR_BF16 = 1 };

/* Scanner geometry (Sec. II; Appendix A).  Projection index i = m N + n with
 * N = rows*cols, view m = floor(i/N), pixel n = row*cols + col.
 * Parallel beam: at theta = 0 rays travel along +x, detector u along +y,
 * v along +z, pixel centre u = (col - (cols-1)/2) pitch_u + off_u,
 * v = (row - (rows-1)/2) pitch_v + off_v.  Cone beam: point source at
 * (-sod, 0, 0), flat detector at x = sdd - sod.  View m rotates the
 * source-detector pair by -theta[m] about z (object rotation by theta[m]) and
 * every sample of the view has time time[m].  The field of view is a box
 * {x0,x1,y0,y1,z0,z1} or a z-axis cylinder {R,z0,z1}; its bounds and [t0,t1]
 * normalise coordinates to [-1,1] (Appendix B item 1).  theta and time are
 * host arrays of n_views entries, copied by dinr_create. */
typedef struct {
  int32_t kind;       /* DINR_PARALLEL or DINR_CONE */
  int32_t rows, cols;
  int32_t n_views;
  int32_t fov_kind;   /* DINR_FOV_BOX or DINR_FOV_CYLINDER */
  int32_t reserved;
  double sod, sdd;
  double pitch_u, pitch_v, off_u, off_v;
  double fov[6];
  double t0, t1;
  const double* theta;
  const double* time;
} dinr_geometry;

/* Coordinate network M(r; gamma) (Appendix B): normalise, Gaussian random
 * Fourier features [cos 2 pi B r; sin 2 pi B r] (2C features), L hidden FC
 * layers of width H with activation `act`, a linear output unit followed by
 * `out_act`.  mu0 scales the field into attenuation units (Eq. (2)).
 * precision: DINR_FP32 runs the MLP GEMMs on FP32 matrix cores; DINR_BF16
 * runs them on BF16 matrix cores with FP32 accumulation.  Supported shapes:
 * (2C, H) in {(128,64), (256,256)}, 1 <= L <= 10, act in {DINR_RELU, DINR_SWISH}
 * (Swish x sigma(x), the activation of the paper's network; its adjoint stashes
 * swish'(z) of every layer, one more H-vector per point and layer). */
typedef struct {
  int32_t n_freq;     /* C */
  int32_t width;      /* H */
  int32_t depth;      /* L */
  int32_t act;
  int32_t out_act;
  int32_t precision;
  int32_t recompute;  /* 1: training steps always run the forward kernel and then a
                         backward kernel that recomputes the activations; 0: when
                         every tile of points holds whole rays (fixed n dividing the
                         tile) the step runs forward, loss and adjoint in one pass */
  int32_t reserved;
  double mu0;
} dinr_mlp;

/* Rays and samples of a projection (Appendix A).  Each projection's pixel is
 * divided into D x D sub-pixels and one ray is traced to the centre of each
 * (sub = D; 0 is read as 1, at most 8).  Samples are equi-spaced midpoints of
 * n equal segments of each ray's chord inside the FOV: mode 0: n fixed;
 * mode 1: n = clamp(ceil(l/h), n_min, n_max) with l the chord length.  The
 * prediction averages mu0 l M over the samples of all D^2 rays, each weighted
 * by its own ray's chord.  A ray missing the FOV has n = 0; a projection none
 * of whose rays hits it is predicted 0.  D > 1 takes the two-pass training
 * step; the query server always traces one ray per pixel with midpoint
 * samples.
 * jitter = 1 places the samples at random (Sec. IV), stratified: sample j of a
 * ray sits at s_in + (j + u) l / n with u uniform in [0, 1), one draw per
 * sample, so the weights are unchanged.  u = (x0 >> 8) 2^-24 with x0 the first
 * word of Philox4x32-10 (Salmon et al., SC'11) of counter (j, k, i mod 2^32,
 * i div 2^32) (k: the ray within projection i) under key (seed, epoch); the
 * epoch is set per call with dinr_set_sample_epoch, so that every training
 * step can draw new positions and any step can be replayed. */
typedef struct {
  int32_t mode;
  int32_t n;
  int32_t n_min, n_max;
  double h;
  int32_t sub;       /* D */
  int32_t jitter;    /* 0 midpoints, 1 stratified random positions */
  uint32_t seed;
  uint32_t reserved;
} dinr_sampling;

/* Adam state for dinr_step (Sec. II, Appendix C).  m_d, v_d: device FP32
 * [n_params], caller-owned, updated in place.  `step` is the 1-based index of
 * this update (bias correction uses beta^step). */
typedef struct {
  float* m_d;
  float* v_d;
  float lr, beta1, beta2, eps;
  int64_t step;
} dinr_adam;

typedef struct dinr_ctx dinr_ctx;

/* Create a context on the current HIP device.  B_host: frozen GRFF matrix,
 * host FP32 [C][4], columns ordered (t, z, y, x) (Appendix B item 2).
 * workspace_budget: bytes of device memory the context may hold.
 * Returns DINR_EINVAL for an unsupported or inconsistent description,
 * DINR_ENOMEM if the budget is below the minimum (a few MB) or cannot be
 * allocated. */
int dinr_create(const dinr_geometry* geom, const dinr_mlp* mlp, const dinr_sampling* samp,
                const float* B_host, size_t workspace_budget, dinr_ctx** out);

int dinr_destroy(dinr_ctx* ctx);

/* Second key word of the random sample positions (sampling.jitter = 1) for
 * the calls enqueued after this one; 0 at creation.  No effect on midpoint
 * sampling.  Returns DINR_EINVAL for a null context. */
int dinr_set_sample_epoch(dinr_ctx* ctx, uint32_t epoch);

/* Message of the last error on this context (static storage of the context). */
const char* dinr_last_error(const dinr_ctx* ctx);

/* Number of parameters of the context's network. */
int64_t dinr_num_params(const dinr_ctx* ctx);

/* Forward projection, Eq. (1)/(7) and Appendix A: for each projection r of
 * the batch, proj_out_d[r] = (1/|Phi_r|) sum_j mu0 l_j M(r_j; gamma) over the
 * samples j of its D^2 rays (l_j: the chord of the ray holding sample j; for
 * D = 1, (1/n_r) sum_j mu0 l_r M(r_{r,j})).
 * params_d: device FP32 [n_params].  proj_idx_d: device int64 [R], each in
 * [0, n_views*rows*cols) (checked on the device: an out-of-range index yields
 * n = 0 and projection NaN).  proj_out_d: device FP32 [R].  n_out_d: device
 * int32 [R] receiving |Phi_r|, the sample count of each projection, or NULL.
 * R D^2 must stay below 2^31 - 1. */
int dinr_forward_project(dinr_ctx* ctx, const float* params_d, const int64_t* proj_idx_d,
                         int64_t R, float* proj_out_d, int32_t* n_out_d, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * projections and counts as dinr_forward_project, bit for bit, with the same
 * arguments, but the call allocates and frees nothing -- its scratch (ray
 * records, offsets, tile map, tile partials, packed weights) is a static
 * 32 MiB device array of the library, not the context's workspace.  That
 * is enough for about 330,000 projections of 256 samples with the
 * 2C = H = 256, six-layer BF16 network (about 96 bytes per ray of 256
 * samples plus the packed weights).  A larger batch is refused with
 * DINR_ENOMEM before anything is enqueued; DINR_EHIP if the array's device
 * address could not be resolved when the context was created.  Every call
 * on a device shares that device's array and leaves the last call's contents
 * in it: calls that overlap in time on one device (from any context or
 * stream) race. */
int dinr_forward_project_noalloc(dinr_ctx* ctx, const float* params_d,
                                 const int64_t* proj_idx_d, int64_t R, float* proj_out_d,
                                 int32_t* n_out_d, void* stream);

/* Adjoint of dinr_forward_project: given dL/dpbar_r in dproj_d (device FP32
 * [R]), writes dL/dgamma = sum_r dproj_r dpbar_r/dgamma (Eq. (8) with an
 * arbitrary upstream) to grad_out_d (device FP32 [n_params], overwritten).
 * gnorm_d (nullable): device double receiving ||grad||^2 computed in FP64. */
int dinr_project_backward(dinr_ctx* ctx, const float* params_d, const int64_t* proj_idx_d,
                          int64_t R, const float* dproj_d, float* grad_out_d, double* gnorm_d,
                          void* stream);

/* One training step on the batch (Eqs. (1), (3), (5), (8)):
 * pbar = forward projection, loss = (1/R) sum_r (meas_r - pbar_r)^2 reduced in
 * FP64, grad = dloss/dgamma (hand-written adjoint; weight gradients summed
 * with FP32 compensated summation), gnorm = ||grad||^2 in FP64.
 * meas_d: device FP32 [R].  proj_out_d (nullable): device FP32 [R].
 * grad_out_d: device FP32 [n_params], overwritten.  loss_d, gnorm_d: device
 * double (nullable).  adam (nullable): when given, params_d is updated in
 * place by one Adam step with the new gradient -- unless the loss or the
 * gradient norm is not finite, which the device checks before updating (the
 * parameters are then left unchanged); dinr_step_status reports it. */
int dinr_step(dinr_ctx* ctx, float* params_d, const int64_t* proj_idx_d, int64_t R,
              const float* meas_d, float* proj_out_d, float* grad_out_d, double* loss_d,
              double* gnorm_d, const dinr_adam* adam, void* stream);

/* Synchronises `stream` and returns DINR_ENONFINITE if the last dinr_step on
 * this context produced a non-finite loss or gradient norm (Adam, if
 * requested, was then skipped), else DINR_OK. */
int dinr_step_status(dinr_ctx* ctx, void* stream);

/* ------------------------------------------------------------------ queries
 * Queries of a trained field (Sec. IV: the network is evaluated on a grid at a
 * view's time, or re-projected): a server keeps the packed weights resident
 * and batches requests continuously on its own stream.
 *  - DINR_QUERY_SLICE: n x n image of mu0 M at height z = z_or_theta (world
 *    units) and time t; pixel (i, j) is at normalised (x, y) =
 *    (-1 + (2j+1)/n, -1 + (2i+1)/n) of the FOV; out[i*n + j].
 *  - DINR_QUERY_REPROJECTION: predicted projections (Eq. (1)) of an n x n
 *    detector with the scanner's geometry kind and detector extent (pitch
 *    scaled by rows/n and cols/n), rotated by theta = z_or_theta, at time t,
 *    with samples_per_ray equi-spaced samples per ray (a divisor of 256 for
 *    BF16 contexts, of 128 for FP32); out[row*n + col], 0 for rays that
 *    miss the FOV. */
enum { DINR_QUERY_SLICE = 0, DINR_QUERY_REPROJECTION = 1 };

typedef struct {
  int32_t kind;
  int32_t n;
  double z_or_theta;
  double t;
  int32_t samples_per_ray;
  int32_t reserved;
} dinr_request;

typedef struct dinr_server dinr_server;

/* Create a query server for `ctx` with the parameters in params_d (device
 * FP32 [n_params]; read at creation to pack the weights and for b_o, so it
 * must stay valid and unchanged while the server lives).  mem_budget bounds
 * the output bytes (4 n^2 per request) of the requests admitted at once;
 * max_active bounds their number.  Starts the scheduler thread.  The server
 * uses its own stream; the context must outlive it and must not be used
 * concurrently for training. */
int dinr_server_create(dinr_ctx* ctx, const float* params_d, size_t mem_budget,
                       int32_t max_active, dinr_server** out);

/* Stops admitting, finishes the requests already admitted, drops queued
 * ones, frees the server. */
int dinr_server_destroy(dinr_server* srv);

/* Submit a request (any thread; never blocks).  out_d: caller-owned device
 * FP32 [n*n], written by the server; valid once dinr_poll reports done.
 * Requests queue in arrival order and are admitted when their output bytes fit
 * in the budget and a slot is free.  DINR_ENOMEM if the request alone exceeds
 * the budget, DINR_EINVAL for a malformed request, DINR_EBUSY once stopped. */
int dinr_query(dinr_server* srv, const dinr_request* req, float* out_d, uint64_t* ticket);

/* done = 1 when the request's output is complete; latency_ms (nullable) gets
 * submit-to-completion time in milliseconds (host clock), or -1. */
int dinr_poll(dinr_server* srv, uint64_t ticket, int32_t* done, double* latency_ms);

/* Block until the request completes (DINR_OK) or the server stops. */
int dinr_query_wait(dinr_server* srv, uint64_t ticket);

/* Forget a completed request's record. */
int dinr_query_release(dinr_server* srv, uint64_t ticket);

/* 4D inference volume (Sec. IV: the trained field voxelised at a list of
 * time instants, written to disk as it is produced).  Voxel (t, k, i, j) is
 * mu0 M at time times[t], height z_k = z0 + (k + 1/2)(z1 - z0)/nz over the FOV's
 * z extent, and slice pixel (i, j) as in DINR_QUERY_SLICE (cell centres of an
 * n x n grid over the FOV's x, y extent).  The file holds a 64-byte header
 * (magic "DINR4DV1", then little-endian int64 nt, nz, n (rows, y), n (columns,
 * x), zero padding), the nt times as float64, then float32 voxels in the order
 * [t][z][y][x].  Slices are computed through the server (sharing it with any
 * other requests), copied to pinned host buffers on a copy stream and written
 * by a writer thread, `slots` slices in flight, so the GPU, the copy engine
 * and the disk overlap. */
typedef struct {
  int32_t n;            /* slice size n x n */
  int32_t nz;           /* slices per time instant */
  int32_t nt;           /* time instants */
  int32_t slots;        /* slices in flight (device and pinned buffers); 0: 4 */
  const double* times;  /* host [nt] */
} dinr_volume;

/* Bytes written, wall-clock seconds of the whole call, and voxels per second
 * (all nullable in the sense that the struct pointer may be NULL). */
typedef struct {
  int64_t bytes;
  double seconds;
  double voxels_per_s;
} dinr_volume_stats;

/* Writes the volume to `path` (created or truncated).  Allocates its slot
 * buffers (4 n^2 bytes each on the device and in pinned host memory) and frees
 * them before returning; blocks until the file is complete.  DINR_EINVAL for
 * a malformed description, DINR_ENOMEM if a slice exceeds the server budget
 * or the buffers cannot be allocated, DINR_EIO if the file cannot be opened or
 * written, DINR_EBUSY if the server stops meanwhile. */
int dinr_volume_write(dinr_server* srv, const dinr_volume* vol, const char* path,
                      dinr_volume_stats* stats);

/* Counters: kernel launches, tiles run, bytes of admitted outputs, queued
 * and admitted requests (all nullable). */
int dinr_server_stats(dinr_server* srv, int64_t* launches, int64_t* tiles, size_t* bytes_in_use,
                      int32_t* queued, int32_t* admitted);

/* Kernel timing (a tracing aid, off by default).  While enabled, every
 * launch of the kernels below is bracketed by a pair of HIP events recorded
 * on the call's stream (at most 4096 launches per kind between reads).
 * dinr_profile_read waits for the recorded events, returns the summed
 * duration in milliseconds and the number of launches of `kind`, and clears
 * them.  Enabling creates the events (host-side HIP objects; no device
 * memory). */
enum {
  DINR_PROF_MLP_FWD = 0,  /* fused forward: coordinates, encoding, MLP, ray-sum */
  DINR_PROF_MLP_BWD = 1,  /* recomputed forward and adjoint chain, operand stash */
  DINR_PROF_WGRAD = 2,    /* weight-gradient reduction over the stash */
  DINR_PROF_MLP_FUSED = 3, /* one-pass forward, ray-sum, loss terms and adjoint chain */
  DINR_PROF_RAYS = 4,     /* ray setup: rays of each projection, offset scan, tile map */
  DINR_PROF_LOSS = 5,     /* residuals, FP64 loss and upstream gradient (with the D x D
                             bundling of ray sums and spreading of the upstream) */
  DINR_PROF_REDUCE = 6,   /* compensated cross-split gradient sums and FP64 ||grad||^2 */
  DINR_PROF_KINDS = 7
};
int dinr_profile_enable(dinr_ctx* ctx, int enable);
int dinr_profile_read(dinr_ctx* ctx, int kind, double* total_ms, int64_t* launches);

/* Sustained BF16 matrix-core rate of the current device (a measurement aid
 * for rooflines, not part of the method).  One workgroup of 8 waves per
 * compute unit; every wave issues `iters` blocks of 16 dependent
 * 32x32x16 BF16 MFMAs.  kind 0: both operands in registers (the matrix
 * pipe's ceiling).  kind 1: the A operand of each MFMA read from LDS, 16
 * bytes per lane, three steps ahead (the operand flow of the MLP layers).
 * Enqueued on `stream` (a hipStream_t, may be null) and waited for; the rate
 * in TFLOP/s goes to *tflops.  Allocates and frees a 4-byte device buffer.
 * Returns DINR_EINVAL for an unknown kind or iters <= 0, DINR_EHIP on a
 * runtime failure. */
int dinr_probe_mfma(int kind, int64_t iters, void* stream, double* tflops);

#ifdef __cplusplus
}
#endif

#endif /* DINR_H */
