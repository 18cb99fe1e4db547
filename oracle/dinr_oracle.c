/*
 * dinr_oracle.c -- plain, slow FP64 CPU reference for the DINR forward model,
 * loss, gradient and Adam update.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file: it exists so that the tests, the smoke check and the CPU baseline
 * of the benchmark can check the GPU path against an independent computation.
 * It shares no code, header, table or constant with the GPU path.
 *
 * Everything is evaluated in IEEE double precision, one ray after another and
 * one sample after another, with no blocking or fusion beyond what the paper's
 * definitions state.  OpenMP splits the rays across threads; per-thread
 * gradient buffers are summed in thread order at the end.
 *
 * Paper being followed (arXiv 2404.19075, "Distributed Stochastic Optimization
 * of a Neural Representation Network for Time-Space Tomography
 * Reconstruction"):
 *   - projection index -> (view m, pixel n): Sec. II, i = mN + n
 *   - rotation of the source-detector pair by -theta, time t_i = T_m: Sec. II
 *   - equi-spaced samples along each ray inside the field of view, weight
 *     w = mu0 * l (chord length in the FOV): Appendix A, Eqs. (1), (2), (7)
 *   - D x D rays per projection, one to the centre of each sub-pixel, and
 *     pbar the average over the samples of all of them: Appendix A
 *   - randomly placed samples along the rays (Sec. IV): optionally, sample j
 *     sits at a uniformly random position inside segment j
 *   - coordinate normalisation to [-1,1], Gaussian random Fourier features
 *     [cos 2 pi B r ; sin 2 pi B r], FC layers, scalar output: Appendix B
 *   - squared distance, local loss, gradient: Eqs. (3), (5), (8)
 *   - Adam: Sec. II and Appendix C
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 *   - parallel beam: at theta = 0 rays travel along +x, detector u = +y,
 *     v = +z; cone beam: source at (-SOD,0,0), flat detector at x = SDD-SOD;
 *     then rotate origin and direction by R_z(-theta_m).
 *   - samples sit at the midpoints of n equal segments of the FOV chord.
 *   - mu0 is applied once, inside w; M itself excludes mu0.
 *   - hidden activation ReLU or Swish; output identity or softplus.
 *   - a ray that misses the FOV has n = 0 and prediction 0.
 *   - with D > 1, |Phi_i| counts the samples of all D^2 rays and each sample
 *     is weighted by the chord length of its own ray.
 *   - random placement is stratified (one sample per segment, so the weights
 *     stay mu0 l / |Phi|); the uniform offset u of sample j of ray k of
 *     projection i comes from Philox4x32-10 (Salmon et al., SC'11) with key
 *     (seed, epoch) and counter (j, k, i mod 2^32, i div 2^32): u = (x0 >> 8) 2^-24
 *     of the first output word, so both implementations draw the same u.
 *
 * Parameter layout (flat, FP64 here): for l = 1..L: W_l [H x fan_in]
 * row-major (row = output unit), b_l [H]; then w_o [H], b_o [1].
 * fan_in is 2C for l = 1 and H otherwise.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

typedef struct {
  int32_t kind;           /* 0 parallel beam, 1 cone beam */
  int32_t rows, cols;     /* detector rows (v) and columns (u) */
  int32_t n_views;
  int32_t fov_kind;       /* 0 box {x0,x1,y0,y1,z0,z1}, 1 cylinder {R,z0,z1} */
  int32_t pad_;
  double sod, sdd;        /* cone beam only */
  double pitch_u, pitch_v, off_u, off_v;
  double fov[6];
  double t0, t1;          /* time normalisation range */
  const double* theta;    /* [n_views] radians */
  const double* time;     /* [n_views] */
} orc_geom;

typedef struct {
  int32_t n_freq;   /* C: encoding has 2C features */
  int32_t width;    /* H */
  int32_t depth;    /* L hidden layers */
  int32_t act;      /* 0 ReLU, 1 Swish */
  int32_t out_act;  /* 0 identity, 1 softplus */
  int32_t pad_;
  double mu0;
} orc_mlp;

typedef struct {
  int32_t mode;     /* 0 fixed n per ray, 1 n = clamp(ceil(l/h), n_min, n_max) */
  int32_t n;
  int32_t n_min, n_max;
  double h;
  int32_t sub;      /* D: rays per projection D x D (0 is read as 1; at most 16) */
  int32_t jitter;   /* 1: stratified random positions instead of midpoints */
  uint32_t seed;    /* first key word of the position generator */
  uint32_t epoch;   /* second key word: one value per training step */
} orc_sampling;

/* Analytic replacement fields used to pin the geometry and the quadrature.
 * kind 0: the MLP.  kind 1: affine in the normalised coordinates,
 * data = {a0, at, az, ay, ax}.  kind 2: moving, deforming ellipsoids in world
 * coordinates, 20 doubles each = {c[3], v[3], s[3], kappa, a, R[9] row-major};
 * at time t the centre is c + v t, the semi-axes s (1 + kappa t), and a point x
 * is inside when |diag(1/s) R^T (x - c)| <= 1; the field is a/mu0 inside.
 * kind 3: moving Gaussian blobs, 8 doubles each = {c[3], v[3], sigma, a};
 * field = a exp(-|x - c - v t|^2 / (2 sigma^2)) / mu0. */
typedef struct {
  int32_t kind;
  int32_t n_items;
  const double* data;
} orc_field;

/* ---------------------------------------------------------------- geometry */

/* Ray k of projection index i (Sec. II, Appendix A): view m = floor(i/N),
 * pixel n = i mod N, row = n / cols, col = n mod cols; the pixel is divided
 * into D x D sub-pixels and ray k = b D + a ends at the centre of sub-pixel
 * (row b, column a).  Returns 0, or -1 for an index out of range.  d is a unit
 * vector, so the ray parameter s is a length. */
int orc_subray(const orc_geom* g, int64_t i, int32_t D, int32_t k, double o[3], double d[3],
               double* t) {
  const int64_t N = (int64_t)g->rows * g->cols;
  if (i < 0 || i >= N * g->n_views || D < 1 || k < 0 || k >= D * D) return -1;
  const int64_t m = i / N;
  const int64_t n = i % N;
  const int64_t row = n / g->cols;
  const int64_t col = n % g->cols;
  const double fa = (k % D + 0.5) / D - 0.5, fb = (k / D + 0.5) / D - 0.5;
  const double u = ((double)col + fa - 0.5 * (g->cols - 1)) * g->pitch_u + g->off_u;
  const double v = ((double)row + fb - 0.5 * (g->rows - 1)) * g->pitch_v + g->off_v;
  double o0[3], d0[3];
  if (g->kind == 0) {
    o0[0] = 0.0; o0[1] = u; o0[2] = v;
    d0[0] = 1.0; d0[1] = 0.0; d0[2] = 0.0;
  } else {
    o0[0] = -g->sod; o0[1] = 0.0; o0[2] = 0.0;
    const double px = g->sdd - g->sod;
    const double ex = px - o0[0], ey = u, ez = v;
    const double nrm = sqrt(ex * ex + ey * ey + ez * ez);
    d0[0] = ex / nrm; d0[1] = ey / nrm; d0[2] = ez / nrm;
  }
  /* rotating the object by theta equals rotating source and detector by
   * -theta about z: R_z(-theta) = [[c, s, 0], [-s, c, 0], [0, 0, 1]] */
  const double th = g->theta[m];
  const double c = cos(th), s = sin(th);
  o[0] = c * o0[0] + s * o0[1];
  o[1] = -s * o0[0] + c * o0[1];
  o[2] = o0[2];
  d[0] = c * d0[0] + s * d0[1];
  d[1] = -s * d0[0] + c * d0[1];
  d[2] = d0[2];
  *t = g->time[m];
  return 0;
}

/* The single ray to the centre of pixel i (D = 1). */
int orc_ray(const orc_geom* g, int64_t i, double o[3], double d[3], double* t) {
  return orc_subray(g, i, 1, 0, o, d, t);
}

static int32_t sub_of(const orc_sampling* s) { return s->sub > 1 ? s->sub : 1; }

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications with the
 * round constants 0xD2511F53 and 0xCD9E8D57, the key bumped by the Weyl
 * constants 0x9E3779B9 and 0xBB67AE85 between rounds. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * x0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    x0 = hi1 ^ x1 ^ k0;
    x1 = lo1;
    x2 = hi0 ^ x3 ^ k1;
    x3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Position of sample j inside its segment, in [0, 1): 1/2 (the midpoint), or
 * the stratified random offset of sample j of ray k of projection i. */
double orc_offset(const orc_sampling* s, int64_t i, int32_t k, int32_t j) {
  if (!s->jitter) return 0.5;
  const uint32_t ctr[4] = {(uint32_t)j, (uint32_t)k, (uint32_t)((uint64_t)i & 0xFFFFFFFFu),
                           (uint32_t)((uint64_t)i >> 32)};
  const uint32_t key[2] = {s->seed, s->epoch};
  uint32_t x[4];
  orc_philox4x32_10(ctr, key, x);
  return (double)(x[0] >> 8) * (1.0 / 16777216.0);
}

/* Chord of the ray inside the field of view: entry parameter and length.
 * Box: slab intersection.  Cylinder about z: quadratic in x,y plus a z slab.
 * A miss gives length 0. */
void orc_clip(const orc_geom* g, const double o[3], const double d[3], double* s_in,
              double* len) {
  double lo = -INFINITY, hi = INFINITY;
  if (g->fov_kind == 0) {
    for (int a = 0; a < 3; ++a) {
      const double b0 = g->fov[2 * a], b1 = g->fov[2 * a + 1];
      if (d[a] == 0.0) {
        if (o[a] < b0 || o[a] > b1) { *s_in = 0.0; *len = 0.0; return; }
      } else {
        double ta = (b0 - o[a]) / d[a], tb = (b1 - o[a]) / d[a];
        if (ta > tb) { const double tmp = ta; ta = tb; tb = tmp; }
        if (ta > lo) lo = ta;
        if (tb < hi) hi = tb;
      }
    }
  } else {
    const double R = g->fov[0], z0 = g->fov[1], z1 = g->fov[2];
    const double qa = d[0] * d[0] + d[1] * d[1];
    const double qb = 2.0 * (o[0] * d[0] + o[1] * d[1]);
    const double qc = o[0] * o[0] + o[1] * o[1] - R * R;
    if (qa == 0.0) {
      if (qc > 0.0) { *s_in = 0.0; *len = 0.0; return; }
    } else {
      const double disc = qb * qb - 4.0 * qa * qc;
      if (disc <= 0.0) { *s_in = 0.0; *len = 0.0; return; }
      const double sq = sqrt(disc);
      lo = (-qb - sq) / (2.0 * qa);
      hi = (-qb + sq) / (2.0 * qa);
    }
    if (d[2] == 0.0) {
      if (o[2] < z0 || o[2] > z1) { *s_in = 0.0; *len = 0.0; return; }
    } else {
      double ta = (z0 - o[2]) / d[2], tb = (z1 - o[2]) / d[2];
      if (ta > tb) { const double tmp = ta; ta = tb; tb = tmp; }
      if (ta > lo) lo = ta;
      if (tb < hi) hi = tb;
    }
  }
  if (hi > lo) { *s_in = lo; *len = hi - lo; }
  else { *s_in = 0.0; *len = 0.0; }
}

/* Number of equi-spaced samples on a chord of length len (Appendix A). */
int32_t orc_nsamp(const orc_sampling* s, double len) {
  if (!(len > 0.0)) return 0;
  if (s->mode == 0) return s->n;
  double q = ceil(len / s->h);
  if (q < s->n_min) q = s->n_min;
  if (q > s->n_max) q = s->n_max;
  return (int32_t)q;
}

/* Normalise (x,y,z,t) to [-1,1]^4 with the FOV bounds (Appendix B item 1).
 * Output order is (t, z, y, x), the column order of B. */
void orc_normalize(const orc_geom* g, const double x[3], double t, double rbar[4]) {
  double lo[3], hi[3];
  if (g->fov_kind == 0) {
    for (int a = 0; a < 3; ++a) { lo[a] = g->fov[2 * a]; hi[a] = g->fov[2 * a + 1]; }
  } else {
    lo[0] = lo[1] = -g->fov[0]; hi[0] = hi[1] = g->fov[0];
    lo[2] = g->fov[1]; hi[2] = g->fov[2];
  }
  rbar[0] = 2.0 * (t - g->t0) / (g->t1 - g->t0) - 1.0;
  rbar[1] = 2.0 * (x[2] - lo[2]) / (hi[2] - lo[2]) - 1.0;
  rbar[2] = 2.0 * (x[1] - lo[1]) / (hi[1] - lo[1]) - 1.0;
  rbar[3] = 2.0 * (x[0] - lo[0]) / (hi[0] - lo[0]) - 1.0;
}

/* ------------------------------------------------------------------ the MLP */

int64_t orc_nparams(const orc_mlp* m) {
  const int64_t C2 = 2 * (int64_t)m->n_freq, H = m->width;
  return H * C2 + H + (int64_t)(m->depth - 1) * (H * H + H) + H + 1;
}

static double act_f(int act, double z) {
  if (act == 0) return z > 0.0 ? z : 0.0;
  return z / (1.0 + exp(-z));
}
static double act_d(int act, double z) {
  if (act == 0) return z > 0.0 ? 1.0 : 0.0;
  const double sg = 1.0 / (1.0 + exp(-z));
  return sg * (1.0 + z * (1.0 - sg));
}
static double out_f(int oa, double z) {
  if (oa == 0) return z;
  return (z > 0.0 ? z : 0.0) + log1p(exp(-fabs(z)));
}
static double out_d(int oa, double z) {
  if (oa == 0) return 1.0;
  return 1.0 / (1.0 + exp(-z));
}

/* Gaussian random Fourier features (Appendix B item 2): u = B rbar,
 * phi = [cos(2 pi u_1..C), sin(2 pi u_1..C)].  B is C x 4 row-major with
 * columns ordered (t, z, y, x). */
static void grff(const orc_mlp* m, const double* B, const double rbar[4], double* phi) {
  const int C = m->n_freq;
  for (int c = 0; c < C; ++c) {
    const double u = B[4 * c + 0] * rbar[0] + B[4 * c + 1] * rbar[1] +
                     B[4 * c + 2] * rbar[2] + B[4 * c + 3] * rbar[3];
    phi[c] = cos(2.0 * ORC_PI * u);
    phi[C + c] = sin(2.0 * ORC_PI * u);
  }
}

/* Work space of one sample: activations a_0..a_L and pre-activations z_1..z_L. */
typedef struct {
  double* a;   /* (L+1) x maxw */
  double* z;   /* (L+1) x maxw, z[0] unused */
  double* da;  /* maxw */
  double* dn;  /* maxw */
  int maxw;
} orc_ws;

static int ws_init(orc_ws* w, const orc_mlp* m) {
  const int maxw = 2 * m->n_freq > m->width ? 2 * m->n_freq : m->width;
  w->maxw = maxw;
  w->a = (double*)malloc(sizeof(double) * (size_t)(m->depth + 1) * maxw);
  w->z = (double*)malloc(sizeof(double) * (size_t)(m->depth + 1) * maxw);
  w->da = (double*)malloc(sizeof(double) * maxw);
  w->dn = (double*)malloc(sizeof(double) * maxw);
  return (w->a && w->z && w->da && w->dn) ? 0 : -1;
}
static void ws_free(orc_ws* w) { free(w->a); free(w->z); free(w->da); free(w->dn); }

/* Forward pass of M(rbar; gamma) (Appendix B).  Fills the work space and
 * returns M; *zo receives the output pre-activation. */
static double mlp_forward(const orc_mlp* m, const double* B, const double* P,
                          const double rbar[4], orc_ws* w, double* zo) {
  const int C2 = 2 * m->n_freq, H = m->width, L = m->depth, mw = w->maxw;
  grff(m, B, rbar, w->a);
  const double* p = P;
  int fin = C2;
  for (int l = 1; l <= L; ++l) {
    const double* W = p;
    const double* b = p + (size_t)H * fin;
    const double* x = w->a + (size_t)(l - 1) * mw;
    double* z = w->z + (size_t)l * mw;
    double* y = w->a + (size_t)l * mw;
    for (int r = 0; r < H; ++r) {
      double s = b[r];
      for (int k = 0; k < fin; ++k) s += W[(size_t)r * fin + k] * x[k];
      z[r] = s;
      y[r] = act_f(m->act, s);
    }
    p += (size_t)H * fin + H;
    fin = H;
  }
  const double* wo = p;
  const double bo = p[H];
  const double* aL = w->a + (size_t)L * mw;
  double s = bo;
  for (int k = 0; k < H; ++k) s += wo[k] * aL[k];
  *zo = s;
  return out_f(m->out_act, s);
}

/* Reverse mode of one sample: adds dM * dM/dgamma to grad.  Needs the work
 * space filled by mlp_forward for the same sample. */
static void mlp_backward(const orc_mlp* m, const double* P, orc_ws* w, double zo,
                         double dM, double* grad) {
  const int C2 = 2 * m->n_freq, H = m->width, L = m->depth, mw = w->maxw;
  /* offsets of each layer's block in the flat layout */
  size_t off[64];
  size_t o = 0;
  int fin = C2;
  for (int l = 1; l <= L; ++l) { off[l] = o; o += (size_t)H * fin + H; fin = H; }
  const size_t off_o = o;
  const double d_o = dM * out_d(m->out_act, zo);
  const double* aL = w->a + (size_t)L * mw;
  for (int k = 0; k < H; ++k) grad[off_o + k] += d_o * aL[k];
  grad[off_o + H] += d_o;
  /* da = dL/da_L */
  for (int k = 0; k < H; ++k) w->da[k] = d_o * P[off_o + k];
  for (int l = L; l >= 1; --l) {
    const int fl = (l == 1) ? C2 : H;
    const double* z = w->z + (size_t)l * mw;
    const double* x = w->a + (size_t)(l - 1) * mw;
    const double* W = P + off[l];
    double* gW = grad + off[l];
    double* gb = grad + off[l] + (size_t)H * fl;
    /* delta_l = da ⊙ act'(z_l), reusing da */
    for (int r = 0; r < H; ++r) w->da[r] *= act_d(m->act, z[r]);
    for (int r = 0; r < H; ++r) {
      const double dr = w->da[r];
      for (int k = 0; k < fl; ++k) gW[(size_t)r * fl + k] += dr * x[k];
      gb[r] += dr;
    }
    if (l > 1) {
      for (int k = 0; k < fl; ++k) {
        double s = 0.0;
        for (int r = 0; r < H; ++r) s += W[(size_t)r * fl + k] * w->da[r];
        w->dn[k] = s;
      }
      memcpy(w->da, w->dn, sizeof(double) * (size_t)fl);
    }
  }
}

/* Field value at a normalised coordinate and world position (x, t). */
static double field_eval(const orc_mlp* m, const orc_field* f, const double* B,
                         const double* P, const double x[3], double t,
                         const double rbar[4], orc_ws* w, double* zo) {
  if (f == NULL || f->kind == 0) return mlp_forward(m, B, P, rbar, w, zo);
  *zo = 0.0;
  if (f->kind == 1) {
    const double* a = f->data;
    return a[0] + a[1] * rbar[0] + a[2] * rbar[1] + a[3] * rbar[2] + a[4] * rbar[3];
  }
  double acc = 0.0;
  if (f->kind == 2) {
    for (int e = 0; e < f->n_items; ++e) {
      const double* q = f->data + 20 * e;
      const double dx = x[0] - (q[0] + q[3] * t);
      const double dy = x[1] - (q[1] + q[4] * t);
      const double dz = x[2] - (q[2] + q[5] * t);
      const double* R = q + 11;
      double r2 = 0.0;
      for (int k = 0; k < 3; ++k) {
        /* (R^T dx)_k = sum_j R[j][k] dx_j */
        const double pk = R[0 * 3 + k] * dx + R[1 * 3 + k] * dy + R[2 * 3 + k] * dz;
        const double sk = q[6 + k] * (1.0 + q[9] * t);
        r2 += (pk / sk) * (pk / sk);
      }
      if (r2 <= 1.0) acc += q[10];
    }
    return acc / m->mu0;
  }
  for (int e = 0; e < f->n_items; ++e) {
    const double* q = f->data + 8 * e;
    const double dx = x[0] - (q[0] + q[3] * t);
    const double dy = x[1] - (q[1] + q[4] * t);
    const double dz = x[2] - (q[2] + q[5] * t);
    acc += q[7] * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * q[6] * q[6]));
  }
  return acc / m->mu0;
}

static int set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  return omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

/* One projection: the D^2 rays of its pixel with n_k samples each, and
 * pbar = (1/|Phi|) sum_k sum_j mu0 l_k M(r_kj), |Phi| = sum_k n_k
 * (Eqs. (1), (2), (7), Appendix A).  n_forced (nullable) holds the D^2 sample
 * counts to use; n_used, s_in_o, len_o receive the D^2 rays' values.
 * Returns -1 on a bad index. */
static int ray_predict(const orc_geom* g, const orc_mlp* m, const orc_sampling* sp,
                       const orc_field* f, const double* B, const double* P, int64_t idx,
                       const int32_t* n_forced, orc_ws* w, double* proj, int32_t* n_used,
                       double* s_in_o, double* len_o) {
  const int32_t D = sub_of(sp);
  double acc = 0.0;  /* sum over rays of l_k sum_j M */
  int64_t n_all = 0;
  for (int32_t k = 0; k < D * D; ++k) {
    double o[3], d[3], t, s_in, len;
    if (orc_subray(g, idx, D, k, o, d, &t) != 0) return -1;
    orc_clip(g, o, d, &s_in, &len);
    int32_t n = n_forced ? n_forced[k] : orc_nsamp(sp, len);
    if (!(len > 0.0)) n = 0;
    double sum = 0.0;
    for (int32_t j = 0; j < n; ++j) {
      const double s = s_in + (j + orc_offset(sp, idx, k, j)) * len / n;
      const double x[3] = {o[0] + s * d[0], o[1] + s * d[1], o[2] + s * d[2]};
      double rbar[4], zo;
      orc_normalize(g, x, t, rbar);
      sum += field_eval(m, f, B, P, x, t, rbar, w, &zo);
    }
    acc += len * sum;
    n_all += n;
    n_used[k] = n;
    s_in_o[k] = s_in;
    len_o[k] = len;
  }
  *proj = (n_all > 0) ? m->mu0 * acc / (double)n_all : 0.0;
  return 0;
}

/* Forward projection of a batch of R projections.  n_override (nullable)
 * forces the per-ray sample counts; proj is [R]; n_override, n_out, s_in_out,
 * len_out are [R D^2], ray k of projection r at r D^2 + k (the last three
 * nullable).  Returns 0, or -1 on a bad index or allocation failure. */
int orc_forward(const orc_geom* g, const orc_mlp* m, const orc_sampling* sp,
                const orc_field* f, const double* B, const double* P, const int64_t* idx,
                int64_t R, const int32_t* n_override, double* proj, int32_t* n_out,
                double* s_in_out, double* len_out, int nthreads) {
  set_threads(nthreads);
  int err = 0;
#pragma omp parallel
  {
    orc_ws w;
    if (ws_init(&w, m) != 0) {
#pragma omp atomic write
      err = -1;
    } else {
#pragma omp for schedule(dynamic, 4)
      for (int64_t r = 0; r < R; ++r) {
        const int32_t D2 = sub_of(sp) * sub_of(sp);
        double p, si[16 * 16], ln[16 * 16];
        int32_t n[16 * 16];
        if (D2 > 16 * 16 ||
            ray_predict(g, m, sp, f, B, P, idx[r], n_override ? n_override + r * D2 : NULL,
                        &w, &p, n, si, ln) != 0) {
#pragma omp atomic write
          err = -1;
          continue;
        }
        proj[r] = p;
        for (int32_t k = 0; k < D2; ++k) {
          if (n_out) n_out[r * D2 + k] = n[k];
          if (s_in_out) s_in_out[r * D2 + k] = si[k];
          if (len_out) len_out[r * D2 + k] = ln[k];
        }
      }
    }
    ws_free(&w);
  }
  return err;
}

/* One training step's loss and gradient (Eqs. (3), (5), (8)) with the MLP
 * field:  L = (1/R) sum_i (p_i - pbar_i)^2,
 *         dL/dgamma = (1/R) sum_i 2 (pbar_i - p_i) (1/|Phi_i|) sum_j mu0 l_ij dM_ij/dgamma,
 * the samples j of projection i spanning its D^2 rays (l_ij: the chord of the
 * ray holding sample j).  n_override (nullable) is [R D^2].
 * grad is [nparams] and is overwritten.  proj (nullable) receives pbar. */
int orc_step(const orc_geom* g, const orc_mlp* m, const orc_sampling* sp, const double* B,
             const double* P, const int64_t* idx, int64_t R, const double* meas,
             const int32_t* n_override, double* proj, double* grad, double* loss,
             int nthreads) {
  if (m->depth < 1 || m->depth > 62) return -1;
  const int nt = set_threads(nthreads);
  const int64_t np = orc_nparams(m);
  double* part = (double*)calloc((size_t)nt * (size_t)np, sizeof(double));
  double* lpart = (double*)calloc((size_t)nt, sizeof(double));
  if (!part || !lpart) { free(part); free(lpart); return -1; }
  int err = 0;
#pragma omp parallel
  {
#ifdef _OPENMP
    const int tid = omp_get_thread_num();
#else
    const int tid = 0;
#endif
    double* gl = part + (size_t)tid * np;
    orc_ws w;
    if (ws_init(&w, m) != 0) {
#pragma omp atomic write
      err = -1;
    } else {
#pragma omp for schedule(dynamic, 4)
      for (int64_t r = 0; r < R; ++r) {
        const int32_t D = sub_of(sp), D2 = D * D;
        /* the D^2 rays of projection r: pbar first, then the adjoint */
        double acc = 0.0;
        int64_t n_all = 0;
        int bad = D2 > 16 * 16;
        for (int32_t k = 0; k < D2 && !bad; ++k) {
          double o[3], d[3], t, s_in, len;
          if (orc_subray(g, idx[r], D, k, o, d, &t) != 0) { bad = 1; break; }
          orc_clip(g, o, d, &s_in, &len);
          int32_t n = n_override ? n_override[r * D2 + k] : orc_nsamp(sp, len);
          if (!(len > 0.0)) n = 0;
          double sum = 0.0;
          for (int32_t j = 0; j < n; ++j) {
            const double s = s_in + (j + orc_offset(sp, idx[r], k, j)) * len / n;
            const double x[3] = {o[0] + s * d[0], o[1] + s * d[1], o[2] + s * d[2]};
            double rbar[4], zo;
            orc_normalize(g, x, t, rbar);
            sum += mlp_forward(m, B, P, rbar, &w, &zo);
          }
          acc += len * sum;
          n_all += n;
        }
        if (bad) {
#pragma omp atomic write
          err = -1;
          continue;
        }
        const double pbar = (n_all > 0) ? m->mu0 * acc / (double)n_all : 0.0;
        if (proj) proj[r] = pbar;
        const double e = meas[r] - pbar;
        lpart[tid] += e * e;
        if (n_all == 0) continue;
        for (int32_t k = 0; k < D2; ++k) {
          double o[3], d[3], t, s_in, len;
          orc_subray(g, idx[r], D, k, o, d, &t);
          orc_clip(g, o, d, &s_in, &len);
          int32_t n = n_override ? n_override[r * D2 + k] : orc_nsamp(sp, len);
          if (!(len > 0.0)) n = 0;
          /* dL/dpbar_i = -2 (p_i - pbar_i) / R ; dpbar_i/dM_kj = mu0 l_k / |Phi_i| */
          const double dM = (-2.0 * e / (double)R) * (m->mu0 * len / (double)n_all);
          for (int32_t j = 0; j < n; ++j) {
            const double s = s_in + (j + orc_offset(sp, idx[r], k, j)) * len / n;
            const double x[3] = {o[0] + s * d[0], o[1] + s * d[1], o[2] + s * d[2]};
            double rbar[4], zo;
            orc_normalize(g, x, t, rbar);
            mlp_forward(m, B, P, rbar, &w, &zo);
            mlp_backward(m, P, &w, zo, dM, gl);
          }
        }
      }
    }
    ws_free(&w);
  }
  if (err == 0) {
    double ls = 0.0;
    for (int k = 0; k < np; ++k) grad[k] = 0.0;
    for (int tt = 0; tt < nt; ++tt) {
      ls += lpart[tt];
      const double* gp = part + (size_t)tt * np;
      for (int64_t k = 0; k < np; ++k) grad[k] += gp[k];
    }
    *loss = ls / (double)R;
  }
  free(part);
  free(lpart);
  return err;
}

/* mu0 * M at world points pts[P][4] = (x, y, z, t), for slice queries
 * (the trained field in LAC units, Sec. IV). */
int orc_field_points(const orc_geom* g, const orc_mlp* m, const double* B, const double* P,
                     const double* pts, int64_t n_pts, double* out, int nthreads) {
  set_threads(nthreads);
  int err = 0;
#pragma omp parallel
  {
    orc_ws w;
    if (ws_init(&w, m) != 0) {
#pragma omp atomic write
      err = -1;
    } else {
#pragma omp for schedule(static)
      for (int64_t k = 0; k < n_pts; ++k) {
        const double x[3] = {pts[4 * k], pts[4 * k + 1], pts[4 * k + 2]};
        double rbar[4], zo;
        orc_normalize(g, x, pts[4 * k + 3], rbar);
        out[k] = m->mu0 * mlp_forward(m, B, P, rbar, &w, &zo);
      }
    }
    ws_free(&w);
  }
  return err;
}

/* Adam with bias correction (the optimiser named in Sec. II and Appendix C);
 * step is the 1-based index of this update. */
void orc_adam(double* p, const double* g, double* mm, double* vv, int64_t n, double lr,
              double b1, double b2, double eps, int64_t step) {
  const double c1 = 1.0 - pow(b1, (double)step);
  const double c2 = 1.0 - pow(b2, (double)step);
  for (int64_t k = 0; k < n; ++k) {
    mm[k] = b1 * mm[k] + (1.0 - b1) * g[k];
    vv[k] = b2 * vv[k] + (1.0 - b2) * g[k] * g[k];
    const double mh = mm[k] / c1, vh = vv[k] / c2;
    p[k] -= lr * mh / (sqrt(vh) + eps);
  }
}

int orc_threads(void) { return set_threads(0); }
