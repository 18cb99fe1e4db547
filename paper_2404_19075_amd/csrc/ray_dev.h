// ray_dev.h -- construction of one detector ray, shared by the ray-setup
// kernel and the query kernel.
#pragma once

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

}  // namespace dinr
