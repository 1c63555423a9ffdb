// Host setup: mesh validation and cell geometry, spatial cell order, the
// direct interaction lists with periodic referred pairs (Sec. 2.2, App. A),
// and the interaction groups that become the GPU work list.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <thread>

#include "aica_internal.h"

namespace aica {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}
const char *last_error_cstr() { return g_err.c_str(); }

int host_threads() {
  const char *e = getenv("AICA_THREADS");
  if (!e) e = getenv("OMP_NUM_THREADS");
  int n = e ? atoi(e) : 0;
  if (n <= 0) n = (int)std::thread::hardware_concurrency();
  if (n <= 0) n = 1;
  return std::min(n, 64);
}


// ------------------------------------------------------------------ small vector helpers

struct V3 {
  double x, y, z;
};
static inline V3 mk(const double *p) { return {p[0], p[1], p[2]}; }
static inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
static inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
static inline V3 operator*(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
static inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

// ------------------------------------------------------------------ referring transforms

Xf Xf::inverse() const {
  Xf v;
  v.rot = rot;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) v.R[3 * i + j] = R[3 * j + i];
  for (int i = 0; i < 3; ++i) v.y[i] = -(v.R[3 * i] * y[0] + v.R[3 * i + 1] * y[1] + v.R[3 * i + 2] * y[2]);
  return v;
}

Xf Xf::then(const Xf &b) const {
  Xf o;
  o.rot = rot || b.rot;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j)
      o.R[3 * i + j] = b.R[3 * i] * R[j] + b.R[3 * i + 1] * R[3 + j] + b.R[3 * i + 2] * R[6 + j];
    o.y[i] = b.R[3 * i] * y[0] + b.R[3 * i + 1] * y[1] + b.R[3 * i + 2] * y[2] + b.y[i];
  }
  return o;
}

Xf image_transform(const Geometry &g, int n0, int n1, int n2) {
  const int n[3] = {n0, n1, n2};
  Xf t;
  for (int k = 0; k < g.nper; ++k) {
    const Xf step = n[k] < 0 ? g.gen[k].inverse() : g.gen[k];
    for (int r = 0; r < std::abs(n[k]); ++r) t = t.then(step);
  }
  if (!t.rot)  // a pure translation: keep the exact sum of the lattice vectors
    for (int q = 0; q < 3; ++q) {
      t.y[q] = 0;
      for (int k = 0; k < g.nper; ++k) t.y[q] += n[k] * g.per[k][q];
    }
  return t;
}

static bool same_xf(const Xf &a, const Xf &b, double scale) {
  for (int i = 0; i < 9; ++i)
    if (std::fabs(a.R[i] - b.R[i]) > 1e-12) return false;
  for (int q = 0; q < 3; ++q)
    if (std::fabs(a.y[q] - b.y[q]) > 1e-9 * scale) return false;
  return true;
}

// Validate the periodic directions' transforms (the rules stated with aica_mesh.periodic_rot).
static int set_transforms(const aica_mesh *m, Geometry &g) {
  double scale = 1.0;
  for (int k = 0; k < g.nper; ++k)
    for (int q = 0; q < 3; ++q) scale += std::fabs(g.per[k][q]);
  for (int k = 0; k < g.nper; ++k) {
    Xf &t = g.gen[k];
    for (int q = 0; q < 3; ++q) t.y[q] = g.per[k][q];
    if (m->periodic_rot) {
      for (int i = 0; i < 9; ++i) {
        t.R[i] = m->periodic_rot[9 * k + i];
        if (!std::isfinite(t.R[i])) return fail(AICA_E_INVAL, "non-finite periodic rotation");
        if (t.R[i] != ((i % 4 == 0) ? 1.0 : 0.0)) t.rot = true;
      }
    }
    g.order[k] = 0;
    if (!t.rot) continue;
    g.has_rot = true;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        const double d = t.R[3 * i] * t.R[3 * j] + t.R[3 * i + 1] * t.R[3 * j + 1] + t.R[3 * i + 2] * t.R[3 * j + 2];
        if (std::fabs(d - (i == j ? 1.0 : 0.0)) > 1e-12) return fail(AICA_E_INVAL, "periodic rotation is not orthonormal");
      }
    const double det = t.R[0] * (t.R[4] * t.R[8] - t.R[5] * t.R[7]) - t.R[1] * (t.R[3] * t.R[8] - t.R[5] * t.R[6]) +
                       t.R[2] * (t.R[3] * t.R[7] - t.R[4] * t.R[6]);
    if (!(det > 0)) return fail(AICA_E_INVAL, "periodic rotation has determinant -1 (a reflection)");
    const Xf id;
    Xf p = t;
    int K = 1;
    while (!same_xf(p, id, scale)) {
      if (++K > 64) return fail(AICA_E_INVAL, "periodic transform with a rotation is not of finite order <= 64");
      p = p.then(t);
    }
    if (K < 3) return fail(AICA_E_INVAL, "periodic transform equals its own inverse (order 2)");
    g.order[k] = K;
  }
  for (int k = 0; k < g.nper; ++k) {
    const V3 a = mk(g.per[k]);
    if (!g.gen[k].rot && !(dot(a, a) > 0)) return fail(AICA_E_INVAL, "zero periodic vector");
    for (int l = 0; l < k; ++l) {
      const V3 b = mk(g.per[l]);
      if (!g.gen[k].rot && !g.gen[l].rot && std::fabs(dot(a, b)) > 1e-12 * std::sqrt(dot(a, a) * dot(b, b)))
        return fail(AICA_E_INVAL, "periodic vectors must be mutually orthogonal");
      if (!same_xf(g.gen[k].then(g.gen[l]), g.gen[l].then(g.gen[k]), scale))
        return fail(AICA_E_INVAL, "the periodic transforms do not commute");
    }
  }
  // the first powers must give distinct images
  int nimg = 1;
  for (int k = 0; k < g.nper; ++k) nimg *= 3;
  std::vector<Xf> im;
  for (int i = 0; i < nimg; ++i) {
    int n[3] = {0, 0, 0}, r = i;
    for (int k = 0; k < g.nper; ++k) {
      n[k] = r % 3 - 1;
      r /= 3;
    }
    im.push_back(image_transform(g, n[0], n[1], n[2]));
    for (int j = 0; j < i; ++j)
      if (same_xf(im[i], im[j], scale)) return fail(AICA_E_INVAL, "two periodic images coincide");
  }
  return AICA_OK;
}

// ------------------------------------------------------------------ geometry

int build_geometry(const aica_mesh *m, Geometry &g) {
  if (!m) return fail(AICA_E_INVAL, "mesh is NULL");
  if (m->n_points <= 0 || m->n_faces <= 0 || m->n_cells <= 0 || !m->points || !m->face_off || !m->face_pts ||
      !m->owner || !m->neighbour)
    return fail(AICA_E_INVAL, "mesh has empty or NULL arrays");
  if (m->n_cells >= (1LL << 31) || m->n_points >= (1LL << 31)) return fail(AICA_E_INVAL, "mesh too large for int32 ids");
  if (m->n_periodic < 0 || m->n_periodic > 3) return fail(AICA_E_INVAL, "n_periodic must be 0..3");
  g.np = m->n_points;
  g.nf = m->n_faces;
  g.nc = m->n_cells;
  g.nper = m->n_periodic;
  for (int k = 0; k < 3; ++k)
    for (int q = 0; q < 3; ++q) g.per[k][q] = k < g.nper ? m->periodic_vec[k][q] : 0.0;
  for (int k = 0; k < g.nper; ++k)
    for (int q = 0; q < 3; ++q)
      if (!std::isfinite(g.per[k][q])) return fail(AICA_E_INVAL, "non-finite periodic vector");
  {
    const int rc = set_transforms(m, g);
    if (rc) return rc;
  }
  g.pts.assign(m->points, m->points + 3 * g.np);
  for (double v : g.pts)
    if (!std::isfinite(v)) return fail(AICA_E_MESH, "non-finite mesh point");
  g.foff.assign(m->face_off, m->face_off + g.nf + 1);
  if (g.foff[0] != 0) return fail(AICA_E_MESH, "face_off[0] must be 0");
  for (int64_t f = 0; f < g.nf; ++f)
    if (g.foff[f + 1] - g.foff[f] < 3) return fail(AICA_E_MESH, "face with fewer than 3 vertices: " + std::to_string(f));
  g.fpts.assign(m->face_pts, m->face_pts + g.foff[g.nf]);
  for (int32_t p : g.fpts)
    if (p < 0 || p >= g.np) return fail(AICA_E_MESH, "face vertex index out of range");
  g.own.assign(m->owner, m->owner + g.nf);
  g.nei.assign(m->neighbour, m->neighbour + g.nf);
  std::vector<int64_t> cnt(g.nc + 1, 0);
  for (int64_t f = 0; f < g.nf; ++f) {
    if (g.own[f] < 0 || g.own[f] >= g.nc) return fail(AICA_E_MESH, "owner out of range");
    if (g.nei[f] < -1 || g.nei[f] >= g.nc || g.nei[f] == g.own[f]) return fail(AICA_E_MESH, "neighbour out of range");
    cnt[g.own[f] + 1]++;
    if (g.nei[f] >= 0) cnt[g.nei[f] + 1]++;
  }
  for (int64_t c = 0; c < g.nc; ++c) {
    if (cnt[c + 1] < 4) return fail(AICA_E_MESH, "cell with fewer than 4 faces: " + std::to_string(c));
    cnt[c + 1] += cnt[c];
  }
  g.cf_off = cnt;
  g.cf.assign(g.cf_off[g.nc], 0);
  g.cf_sgn.assign(g.cf_off[g.nc], 0);
  {
    std::vector<int64_t> fill(g.cf_off.begin(), g.cf_off.end() - 1);
    for (int64_t f = 0; f < g.nf; ++f) {
      int64_t k = fill[g.own[f]]++;
      g.cf[k] = (int32_t)f;
      g.cf_sgn[k] = 1;
      if (g.nei[f] >= 0) {
        k = fill[g.nei[f]]++;
        g.cf[k] = (int32_t)f;
        g.cf_sgn[k] = -1;
      }
    }
  }
  g.fcen.assign(3 * g.nf, 0.0);
  parallel_for(g.nf, [&](int64_t b, int64_t e, int) {
    for (int64_t f = b; f < e; ++f) {
      double s[3] = {0, 0, 0};
      int64_t len = g.foff[f + 1] - g.foff[f];
      for (int64_t k = g.foff[f]; k < g.foff[f + 1]; ++k)
        for (int q = 0; q < 3; ++q) s[q] += g.pts[3 * (int64_t)g.fpts[k] + q];
      for (int q = 0; q < 3; ++q) g.fcen[3 * f + q] = s[q] / (double)len;
    }
  });
  // distinct vertices per cell
  std::vector<int64_t> vcount(g.nc + 1, 0);
  std::vector<std::vector<int32_t>> tmp;  // only used for sizing via per-thread buffers
  std::vector<int32_t> nverts(g.nc, 0);
  parallel_for(g.nc, [&](int64_t b, int64_t e, int) {
    std::vector<int32_t> ids;
    for (int64_t c = b; c < e; ++c) {
      ids.clear();
      for (int64_t k = g.cf_off[c]; k < g.cf_off[c + 1]; ++k) {
        int32_t f = g.cf[k];
        for (int64_t j = g.foff[f]; j < g.foff[f + 1]; ++j) ids.push_back(g.fpts[j]);
      }
      std::sort(ids.begin(), ids.end());
      nverts[c] = (int32_t)(std::unique(ids.begin(), ids.end()) - ids.begin());
    }
  });
  g.cv_off.assign(g.nc + 1, 0);
  for (int64_t c = 0; c < g.nc; ++c) g.cv_off[c + 1] = g.cv_off[c] + nverts[c];
  g.cv.assign(g.cv_off[g.nc], 0);
  g.ccen.assign(3 * g.nc, 0.0);
  g.lo.assign(3 * g.nc, 0.0);
  g.hi.assign(3 * g.nc, 0.0);
  g.vol.assign(g.nc, 0.0);
  g.r_in.assign(g.nc, 0.0);
  g.r_out.assign(g.nc, 0.0);
  std::vector<int64_t> bad(host_threads() + 1, -1);
  std::atomic<int64_t> first_bad(-1);
  parallel_for(g.nc, [&](int64_t b, int64_t e, int) {
    std::vector<int32_t> ids;
    for (int64_t c = b; c < e; ++c) {
      ids.clear();
      for (int64_t k = g.cf_off[c]; k < g.cf_off[c + 1]; ++k) {
        int32_t f = g.cf[k];
        for (int64_t j = g.foff[f]; j < g.foff[f + 1]; ++j) ids.push_back(g.fpts[j]);
      }
      std::sort(ids.begin(), ids.end());
      ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
      double s[3] = {0, 0, 0}, lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
      for (size_t j = 0; j < ids.size(); ++j) {
        g.cv[g.cv_off[c] + j] = ids[j];
        for (int q = 0; q < 3; ++q) {
          double v = g.pts[3 * (int64_t)ids[j] + q];
          s[q] += v;
          lo[q] = std::min(lo[q], v);
          hi[q] = std::max(hi[q], v);
        }
      }
      for (int q = 0; q < 3; ++q) {
        g.ccen[3 * c + q] = s[q] / (double)ids.size();
        g.lo[3 * c + q] = lo[q];
        g.hi[3 * c + q] = hi[q];
      }
      // tetrahedra (cell centroid, face centroid, edge) must all have positive volume
      V3 cc = mk(&g.ccen[3 * c]);
      double vol = 0, rin = 1e300, rout = 0;
      bool ok = true;
      for (size_t j = 0; j < ids.size(); ++j) {
        V3 v = mk(&g.pts[3 * (int64_t)ids[j]]) - cc;
        rout = std::max(rout, std::sqrt(dot(v, v)));
      }
      for (int64_t k = g.cf_off[c]; k < g.cf_off[c + 1]; ++k) {
        int32_t f = g.cf[k];
        V3 fc = mk(&g.fcen[3 * (int64_t)f]);
        int64_t b0 = g.foff[f], len = g.foff[f + 1] - b0;
        for (int64_t j = 0; j < len; ++j) {
          int64_t ia = g.fpts[b0 + j], ib = g.fpts[b0 + (j + 1) % len];
          if (g.cf_sgn[k] < 0) std::swap(ia, ib);
          V3 a = mk(&g.pts[3 * ia]), bb = mk(&g.pts[3 * ib]);
          double v = dot(fc - cc, cross(a - cc, bb - cc)) / 6.0;
          if (!(v > 0)) ok = false;
          vol += v;
          // distance from the centroid to the plane of the face triangle = 3 V / area
          V3 n = cross(a - fc, bb - fc);
          double area = 0.5 * std::sqrt(dot(n, n));
          if (area > 0) rin = std::min(rin, 3.0 * v / area);
        }
      }
      g.vol[c] = vol;
      // every point within rin of the centroid lies in the cone of some face triangle and on the inner
      // side of that triangle's plane, hence inside the cell
      g.r_in[c] = std::max(0.0, rin) * (1.0 - 1e-12);
      g.r_out[c] = rout * (1.0 + 1e-12);
      if (!ok) {
        int64_t exp = -1;
        first_bad.compare_exchange_strong(exp, c);
      }
    }
  });
  if (first_bad.load() >= 0)
    return fail(AICA_E_MESH, "cell " + std::to_string(first_bad.load()) +
                                 " has a non-positive tetrahedron (inverted, open or misoriented)");
  for (int q = 0; q < 3; ++q) {
    g.dom_lo[q] = 1e300;
    g.dom_hi[q] = -1e300;
    g.max_half_ext[q] = 0;
  }
  g.total_volume = 0;
  for (int64_t c = 0; c < g.nc; ++c) {
    for (int q = 0; q < 3; ++q) {
      g.dom_lo[q] = std::min(g.dom_lo[q], g.lo[3 * c + q]);
      g.dom_hi[q] = std::max(g.dom_hi[q], g.hi[3 * c + q]);
      g.max_half_ext[q] = std::max(g.max_half_ext[q], std::max(g.hi[3 * c + q] - g.ccen[3 * c + q],
                                                               g.ccen[3 * c + q] - g.lo[3 * c + q]));
    }
    g.total_volume += g.vol[c];
  }
  return AICA_OK;
}

// ------------------------------------------------------------------ spatial order

void spatial_order(const Geometry &g, std::vector<int32_t> &order, std::vector<int32_t> &rank,
                   std::vector<uint8_t> &split_depth) {
  order.resize(g.nc);
  std::iota(order.begin(), order.end(), 0);
  // split_depth[s]: depth of the node of the k-d tree that splits its range at sorted position s (every
  // position but 0 splits exactly one node; the root has depth 0)
  split_depth.assign(g.nc, 255);
  struct Range {
    int64_t b, e;
    int depth;
  };
  std::vector<Range> stack{{0, g.nc, 0}};
  while (!stack.empty()) {
    Range r = stack.back();
    stack.pop_back();
    if (r.e - r.b <= 1) continue;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = r.b; i < r.e; ++i)
      for (int q = 0; q < 3; ++q) {
        double v = g.ccen[3 * (int64_t)order[i] + q];
        lo[q] = std::min(lo[q], v);
        hi[q] = std::max(hi[q], v);
      }
    int ax = 0;
    for (int q = 1; q < 3; ++q)
      if (hi[q] - lo[q] > hi[ax] - lo[ax]) ax = q;
    int64_t mid = r.b + (r.e - r.b) / 2;
    std::nth_element(order.begin() + r.b, order.begin() + mid, order.begin() + r.e, [&](int32_t a, int32_t b) {
      double va = g.ccen[3 * (int64_t)a + ax], vb = g.ccen[3 * (int64_t)b + ax];
      return va < vb || (va == vb && a < b);
    });
    split_depth[mid] = (uint8_t)std::min(r.depth, 254);
    // right half pushed first so the left half is processed (and ordered) first
    stack.push_back({mid, r.e, r.depth + 1});
    stack.push_back({r.b, mid, r.depth + 1});
  }
  rank.assign(g.nc, 0);
  for (int64_t s = 0; s < g.nc; ++s) rank[order[s]] = (int32_t)s;
}

// ------------------------------------------------------------------ closest points (published methods)

// Closest point on triangle abc to p: Voronoi-region classification of
// Ericson, Real-Time Collision Detection (2004), Sec. 5.1.5.
static inline V3 closest_on_triangle(V3 p, V3 a, V3 b, V3 c) {
  V3 ab = b - a, ac = c - a, ap = p - a;
  double d1 = dot(ab, ap), d2 = dot(ac, ap);
  if (d1 <= 0 && d2 <= 0) return a;
  V3 bp = p - b;
  double d3 = dot(ab, bp), d4 = dot(ac, bp);
  if (d3 >= 0 && d4 <= d3) return b;
  double vc = d1 * d4 - d3 * d2;
  if (vc <= 0 && d1 >= 0 && d3 <= 0) return a + ab * (d1 / (d1 - d3));
  V3 cp = p - c;
  double d5 = dot(ab, cp), d6 = dot(ac, cp);
  if (d6 >= 0 && d5 <= d6) return c;
  double vb = d5 * d2 - d1 * d6;
  if (vb <= 0 && d2 >= 0 && d6 <= 0) return a + ac * (d2 / (d2 - d6));
  double va = d3 * d6 - d5 * d4;
  if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0) return b + (c - b) * ((d4 - d3) / ((d4 - d3) + (d5 - d6)));
  double den = 1.0 / (va + vb + vc);
  return a + ab * (vb * den) + ac * (vc * den);
}

static inline double clamp01(double v) { return v < 0 ? 0 : (v > 1 ? 1 : v); }

// Squared distance between segments p1q1 and p2q2 (Ericson, Sec. 5.1.9).
static inline double seg_seg_d2(V3 p1, V3 q1, V3 p2, V3 q2) {
  V3 d1 = q1 - p1, d2 = q2 - p2, r = p1 - p2;
  double a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r);
  double s, t;
  const double tiny = 1e-300;
  if (a <= tiny && e <= tiny) return dot(r, r);
  if (a <= tiny) {
    s = 0;
    t = clamp01(f / e);
  } else {
    double c = dot(d1, r);
    if (e <= tiny) {
      t = 0;
      s = clamp01(-c / a);
    } else {
      double b = dot(d1, d2), den = a * e - b * b;
      s = den != 0 ? clamp01((b * f - c * e) / den) : 0.0;
      t = (b * s + f) / e;
      if (t < 0) {
        t = 0;
        s = clamp01(-c / a);
      } else if (t > 1) {
        t = 1;
        s = clamp01((b - c) / a);
      }
    }
  }
  V3 w = (p1 + d1 * s) - (p2 + d2 * t);
  return dot(w, w);
}

// Squared distance between two triangles that do not interpenetrate.
static inline double tri_tri_d2(const V3 *A, const V3 *B, double stop) {
  double best = 1e300;
  for (int i = 0; i < 3; ++i) {
    V3 q = closest_on_triangle(A[i], B[0], B[1], B[2]);
    best = std::min(best, dot(A[i] - q, A[i] - q));
    q = closest_on_triangle(B[i], A[0], A[1], A[2]);
    best = std::min(best, dot(B[i] - q, B[i] - q));
    if (best < stop) return best;
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      best = std::min(best, seg_seg_d2(A[i], A[(i + 1) % 3], B[j], B[(j + 1) % 3]));
      if (best < stop) return best;
    }
  return best;
}

struct CellTris {
  std::vector<V3> t;       // 3 per triangle
  std::vector<double> bb;  // 6 per triangle: lo, hi
};

static inline V3 mapped(const Xf &T, const double *p) {
  double o[3];
  T.apply(p, o);
  return mk(o);
}

static void cell_triangles(const Geometry &g, int32_t c, const Xf &T, CellTris &out) {
  out.t.clear();
  out.bb.clear();
  for (int64_t k = g.cf_off[c]; k < g.cf_off[c + 1]; ++k) {
    int32_t f = g.cf[k];
    V3 fc = mapped(T, &g.fcen[3 * (int64_t)f]);
    int64_t b0 = g.foff[f], len = g.foff[f + 1] - b0;
    for (int64_t j = 0; j < len; ++j) {
      V3 a = mapped(T, &g.pts[3 * (int64_t)g.fpts[b0 + j]]);
      V3 b = mapped(T, &g.pts[3 * (int64_t)g.fpts[b0 + (j + 1) % len]]);
      out.t.push_back(fc);
      out.t.push_back(a);
      out.t.push_back(b);
      out.bb.push_back(std::min({fc.x, a.x, b.x}));
      out.bb.push_back(std::min({fc.y, a.y, b.y}));
      out.bb.push_back(std::min({fc.z, a.z, b.z}));
      out.bb.push_back(std::max({fc.x, a.x, b.x}));
      out.bb.push_back(std::max({fc.y, a.y, b.y}));
      out.bb.push_back(std::max({fc.z, a.z, b.z}));
    }
  }
}

static inline double box_gap2(const double *alo, const double *ahi, const double *blo, const double *bhi) {
  double s = 0;
  for (int q = 0; q < 3; ++q) {
    double gap = 0;
    if (blo[q] > ahi[q]) gap = blo[q] - ahi[q];
    if (alo[q] > bhi[q]) gap = alo[q] - bhi[q];
    s += gap * gap;
  }
  return s;
}

// Is the closest distance between cell c and cell d translated by T below R?
// Compact per-cell bounds in sorted order for the candidate scan.
struct CellBox {
  double lo[3], hi[3], cen[3], rin, rout;
};

// Bounding box of box [lo, hi] mapped by T (the box itself for a translation).
static inline void mapped_box(const Xf &T, const double *lo, const double *hi, double *mlo, double *mhi) {
  if (!T.rot) {
    for (int q = 0; q < 3; ++q) {
      mlo[q] = lo[q] + T.y[q];
      mhi[q] = hi[q] + T.y[q];
    }
    return;
  }
  for (int q = 0; q < 3; ++q) {
    mlo[q] = 1e300;
    mhi[q] = -1e300;
  }
  for (int k = 0; k < 8; ++k) {
    const double p[3] = {(k & 1) ? hi[0] : lo[0], (k & 2) ? hi[1] : lo[1], (k & 4) ? hi[2] : lo[2]};
    double o[3];
    T.apply(p, o);
    for (int q = 0; q < 3; ++q) {
      mlo[q] = std::min(mlo[q], o[q]);
      mhi[q] = std::max(mhi[q], o[q]);
    }
  }
}

// Cheap classification: 1 = in range, 0 = not, -1 = undecided (needs the exact test).
static inline int quick_range(const CellBox &C, const CellBox &D, const Xf &T, double R) {
  const double R2 = R * R;
  double g2 = 0;
  double dlo[3], dhi[3], dc[3];
  mapped_box(T, D.lo, D.hi, dlo, dhi);
  for (int q = 0; q < 3; ++q) {
    double gap = 0;
    if (dlo[q] > C.hi[q]) gap = dlo[q] - C.hi[q];
    if (C.lo[q] > dhi[q]) gap = C.lo[q] - dhi[q];
    g2 += gap * gap;
  }
  if (g2 >= R2) return 0;
  // balls of radius r_in about the centroids lie inside the cells (upper bound on the distance);
  // balls of radius r_out contain them (lower bound)
  T.apply(D.cen, dc);
  const double d0 = C.cen[0] - dc[0], d1 = C.cen[1] - dc[1], d2 = C.cen[2] - dc[2];
  const double cd = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  if (cd - C.rin - D.rin < R) return 1;
  if (cd - C.rout - D.rout >= R) return 0;
  return -1;
}

// Exact test (after quick_range returned -1): vertex pairs, then boundary triangle pairs.
static bool cells_in_range(const Geometry &g, int32_t c, int32_t d, const Xf &T, double R, CellTris &tc,
                           CellTris &td) {
  const double R2 = R * R;
  // d's vertices mapped by T (they span its convex hull, which holds the cell)
  std::vector<V3> &dv = td.t;
  dv.clear();
  double dlo[3] = {1e300, 1e300, 1e300}, dhi[3] = {-1e300, -1e300, -1e300};
  for (int64_t j = g.cv_off[d]; j < g.cv_off[d + 1]; ++j) {
    const V3 b = mapped(T, &g.pts[3 * (int64_t)g.cv[j]]);
    dv.push_back(b);
    const double bq[3] = {b.x, b.y, b.z};
    for (int q = 0; q < 3; ++q) {
      dlo[q] = std::min(dlo[q], bq[q]);
      dhi[q] = std::max(dhi[q], bq[q]);
    }
  }
  // separating axis along the centroid direction: every cell lies in the convex hull of its vertices,
  // so a projection gap of at least R proves the cells are out of range
  {
    V3 u = mapped(T, &g.ccen[3 * (int64_t)d]) - mk(&g.ccen[3 * (int64_t)c]);
    const double uu = std::sqrt(dot(u, u));
    if (uu > 0) {
      u = u * (1.0 / uu);
      double cmax = -1e300, dmin = 1e300;
      for (int64_t i = g.cv_off[c]; i < g.cv_off[c + 1]; ++i) cmax = std::max(cmax, dot(mk(&g.pts[3 * (int64_t)g.cv[i]]), u));
      for (const V3 &b : dv) dmin = std::min(dmin, dot(b, u));
      if (dmin - cmax >= R * (1.0 + 1e-12)) return false;
    }
  }
  for (int64_t i = g.cv_off[c]; i < g.cv_off[c + 1]; ++i) {
    V3 a = mk(&g.pts[3 * (int64_t)g.cv[i]]);
    for (const V3 &b : dv)
      if (dot(a - b, a - b) < R2) return true;
  }
  cell_triangles(g, c, Xf(), tc);
  cell_triangles(g, d, T, td);
  const size_t nt = tc.bb.size() / 6, nd = td.bb.size() / 6;
  for (size_t i = 0; i < nt; ++i) {
    const double *bi = &tc.bb[6 * i];
    if (box_gap2(bi, bi + 3, dlo, dhi) >= R2) continue;
    for (size_t j = 0; j < nd; ++j) {
      const double *bj = &td.bb[6 * j];
      if (box_gap2(bi, bi + 3, bj, bj + 3) >= R2) continue;
      if (tri_tri_d2(&tc.t[3 * i], &td.t[3 * j], R2) < R2) return true;
    }
  }
  return false;
}

static inline int img_code(int n0, int n1, int n2) { return 9 * (n0 + 1) + 3 * (n1 + 1) + (n2 + 1); }

// Closest-distance predicate (predicate AICA_DIL_CLOSEST), or the paper's vertex-to-vertex predicate
// (AICA_DIL_VERTEX: some vertex of c and some vertex of d + T closer than R).
static bool vertices_in_range(const Geometry &g, int32_t c, int32_t d, const Xf &T, double R) {
  const double R2 = R * R;
  for (int64_t i = g.cv_off[c]; i < g.cv_off[c + 1]; ++i) {
    const V3 a = mk(&g.pts[3 * (int64_t)g.cv[i]]);
    for (int64_t j = g.cv_off[d]; j < g.cv_off[d + 1]; ++j) {
      const V3 b = mapped(T, &g.pts[3 * (int64_t)g.cv[j]]);
      if (dot(a - b, a - b) < R2) return true;
    }
  }
  return false;
}

int build_cell_pairs(const Geometry &g, const std::vector<int32_t> &order, const std::vector<int32_t> &rank,
                     double R, int predicate, std::vector<CellPair> &out) {
  for (int k = 0; k < g.nper; ++k) {
    if (g.gen[k].rot) continue;
    double L = std::sqrt(dot(mk(g.per[k]), mk(g.per[k])));
    if (!(R < 0.5 * L))
      return fail(AICA_E_RCUT, "rcut + guard must be below half of every periodic length (" + std::to_string(R) +
                                   " vs " + std::to_string(L) + ")");
  }
  // uniform grid of cell centroids over the mesh bounding box
  // centroid bins about one mean cell size per axis
  double binq[3];
  const double hmean = std::cbrt(g.total_volume / (double)g.nc);
  for (int q = 0; q < 3; ++q) binq[q] = std::max(hmean, 1e-9);
  int64_t nb[3];
  for (int q = 0; q < 3; ++q) nb[q] = std::max<int64_t>(1, (int64_t)std::ceil((g.dom_hi[q] - g.dom_lo[q]) / binq[q]));
  while (nb[0] * nb[1] * nb[2] > 4 * g.nc + 64) {
    for (int q = 0; q < 3; ++q) {
      binq[q] *= 1.25;
      nb[q] = std::max<int64_t>(1, (int64_t)std::ceil((g.dom_hi[q] - g.dom_lo[q]) / binq[q]));
    }
  }
  const int64_t nbins = nb[0] * nb[1] * nb[2];
  const double bin = std::max({binq[0], binq[1], binq[2]});
  auto bin_of = [&](double v, int q) {
    int64_t b = (int64_t)std::floor((v - g.dom_lo[q]) / binq[q]);
    return std::min<int64_t>(std::max<int64_t>(b, 0), nb[q] - 1);
  };
  std::vector<CellBox> box(g.nc);
  for (int64_t s = 0; s < g.nc; ++s) {
    const int64_t c = order[s];
    for (int q = 0; q < 3; ++q) {
      box[s].lo[q] = g.lo[3 * c + q];
      box[s].hi[q] = g.hi[3 * c + q];
      box[s].cen[q] = g.ccen[3 * c + q];
    }
    box[s].rin = g.r_in[c];
    box[s].rout = g.r_out[c];
  }
  std::vector<int64_t> boff(nbins + 1, 0);
  std::vector<int32_t> bcell(g.nc);
  for (int64_t c = 0; c < g.nc; ++c) {
    int64_t b = bin_of(g.ccen[3 * c], 0) + nb[0] * (bin_of(g.ccen[3 * c + 1], 1) + nb[1] * bin_of(g.ccen[3 * c + 2], 2));
    boff[b + 1]++;
  }
  for (int64_t b = 0; b < nbins; ++b) boff[b + 1] += boff[b];
  {
    std::vector<int64_t> fill(boff.begin(), boff.end() - 1);
    for (int64_t s = 0; s < g.nc; ++s) {  // in sorted order so bins list ascending sorted ids
      int64_t c = order[s];
      int64_t b = bin_of(g.ccen[3 * c], 0) + nb[0] * (bin_of(g.ccen[3 * c + 1], 1) + nb[1] * bin_of(g.ccen[3 * c + 2], 2));
      bcell[fill[b]++] = (int32_t)s;  // sorted id
    }
  }
  // images: the first powers (listed pairs); with a rotation also every other power (translations to
  // +-2, rotations over their whole group), which must find no cell pair in range
  struct Img {
    Xf T, Tinv;
    int n[3];
  };
  std::vector<Img> imgs, far;
  {
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int k = 0; k < g.nper; ++k) {
      lo[k] = g.gen[k].rot ? -((g.order[k] - 1) / 2) : -2;
      hi[k] = g.gen[k].rot ? g.order[k] / 2 : 2;
    }
    for (int a = lo[0]; a <= hi[0]; ++a)
      for (int b = lo[1]; b <= hi[1]; ++b)
        for (int c = lo[2]; c <= hi[2]; ++c) {
          Img im;
          im.n[0] = a;
          im.n[1] = b;
          im.n[2] = c;
          im.T = image_transform(g, a, b, c);
          im.Tinv = im.T.inverse();
          const bool first = std::abs(a) <= 1 && std::abs(b) <= 1 && std::abs(c) <= 1;
          if (first) imgs.push_back(im);
          else if (g.has_rot) far.push_back(im);
        }
  }
  const int nt = host_threads();
  std::vector<std::vector<CellPair>> per_thread(nt);
  std::vector<std::vector<CellPair>> per_chunk;
  std::mutex mu;
  // process sorted cells in chunks; each chunk's pairs are sorted afterwards
  const int64_t chunk = 2048;
  const int64_t nchunks = (g.nc + chunk - 1) / chunk;
  per_chunk.resize(nchunks);
  std::atomic<int64_t> next(0), n_cand(0), n_exact(0), n_far(0);
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      CellTris tc, td;
      std::vector<CellPair> local;
      int64_t stat_cand = 0, stat_exact = 0, stat_far = 0;
      for (;;) {
        int64_t ch = next.fetch_add(1);
        if (ch >= nchunks) break;
        local.clear();
        for (int64_t sc = ch * chunk; sc < std::min<int64_t>(g.nc, (ch + 1) * chunk); ++sc) {
          int32_t c = order[sc];
          for (int pass = 0; pass < 2; ++pass)
          for (const Img &im : pass == 0 ? imgs : far) {
            const bool is_far = pass == 1;
            const int *n = im.n;
            const Xf &T = im.T;
            const int code = is_far ? 0 : img_code(n[0], n[1], n[2]);
            // d meets box_c grown by R after T, so its centroid lies within ext of T^-1 of that box
            int64_t b0[3], b1[3];
            bool empty = false;
            double glo[3], ghi[3], qlo[3], qhi[3];
            for (int q = 0; q < 3; ++q) {
              glo[q] = g.lo[3 * (int64_t)c + q] - R;
              ghi[q] = g.hi[3 * (int64_t)c + q] + R;
            }
            mapped_box(im.Tinv, glo, ghi, qlo, qhi);
            for (int q = 0; q < 3; ++q) {
              double lo = qlo[q] - g.max_half_ext[q];
              double hi = qhi[q] + g.max_half_ext[q];
              if (hi < g.dom_lo[q] - bin || lo > g.dom_hi[q] + bin) empty = true;
              b0[q] = bin_of(lo, q);
              b1[q] = bin_of(hi, q);
            }
            if (empty) continue;
            for (int64_t z = b0[2]; z <= b1[2]; ++z)
              for (int64_t y = b0[1]; y <= b1[1]; ++y)
                for (int64_t x = b0[0]; x <= b1[0]; ++x) {
                  int64_t b = x + nb[0] * (y + nb[1] * z);
                  for (int64_t k = boff[b]; k < boff[b + 1]; ++k) {
                    const int32_t sd = bcell[k];
                    if (is_far) {  // any cell pair through a farther image is an error
                      if (quick_range(box[sc], box[sd], T, R) != 0 && cells_in_range(g, c, order[sd], T, R, tc, td))
                        ++stat_far;
                      continue;
                    }
                    if (sd < sc || (sd == sc && code <= 13)) continue;  // canonical half
                    int q = quick_range(box[sc], box[sd], T, R);
                    ++stat_cand;
                    if (predicate == AICA_DIL_VERTEX) {
                      // the bounding boxes hold the vertices: only their gap may decide
                      if (q != 0) {
                        ++stat_exact;
                        q = vertices_in_range(g, c, order[sd], T, R) ? 1 : 0;
                      }
                    } else if (q < 0) {
                      ++stat_exact;
                      q = cells_in_range(g, c, order[sd], T, R, tc, td) ? 1 : 0;
                    }
                    if (q) {
                      CellPair p;
                      p.sc = (int32_t)sc;
                      p.sd = sd;
                      p.img[0] = (int8_t)n[0];
                      p.img[1] = (int8_t)n[1];
                      p.img[2] = (int8_t)n[2];
                      local.push_back(p);
                    }
                  }
                }
          }
        }
        std::sort(local.begin(), local.end(), [](const CellPair &a, const CellPair &b) {
          if (a.sc != b.sc) return a.sc < b.sc;
          if (a.sd != b.sd) return a.sd < b.sd;
          return img_code(a.img[0], a.img[1], a.img[2]) < img_code(b.img[0], b.img[1], b.img[2]);
        });
        per_chunk[ch] = local;
      }
      n_cand += stat_cand;
      n_exact += stat_exact;
      n_far += stat_far;
    });
  for (auto &x : th) x.join();
  if (n_far.load() > 0)
    return fail(AICA_E_RCUT, "rcut + guard reaches " + std::to_string(n_far.load()) +
                                 " cell pairs through images beyond the first power of the periodic transforms");
  if (getenv("AICA_VERBOSE"))
    fprintf(stderr, "cell pairs: %lld candidates, %lld exact tests, %lld bins\n", (long long)n_cand.load(),
            (long long)n_exact.load(), (long long)nbins);
  size_t total = 0;
  for (auto &v : per_chunk) total += v.size();
  out.clear();
  out.reserve(total);
  for (auto &v : per_chunk) {
    out.insert(out.end(), v.begin(), v.end());
    std::vector<CellPair>().swap(v);
  }
  return AICA_OK;
}

// ------------------------------------------------------------------ interaction groups

int build_groups(const Geometry &g, const std::vector<int32_t> &order, const std::vector<uint8_t> &split_depth,
                 const std::vector<CellPair> &pairs, double density, double target, Groups &G) {
  const int64_t nc = g.nc;
  G.cell0.clear();
  G.of_cell.assign(nc, 0);
  // Groups are subtrees of the k-d tree of the sorted order: descending from the root, a subtree whose
  // expected occupancy is at most the target becomes a group, so every group is a compact box-like block
  // of cells (a run of the sorted order cut at arbitrary places would straddle subtrees and spread out).
  std::vector<double> vpre(nc + 1, 0.0);
  for (int64_t s = 0; s < nc; ++s) vpre[s + 1] = vpre[s] + g.vol[order[s]];
  struct Node {
    int64_t b, e;
    int depth;
  };
  std::vector<Node> stack{{0, nc, 0}};
  while (!stack.empty()) {
    const Node r = stack.back();
    stack.pop_back();
    if (r.e <= r.b) continue;
    if (r.e - r.b == 1 || density * (vpre[r.e] - vpre[r.b]) <= target) {
      G.cell0.push_back((int32_t)r.b);
      continue;
    }
    int64_t mid = r.b + 1;
    while (mid < r.e && split_depth[mid] != (uint8_t)std::min(r.depth, 254)) ++mid;
    if (mid >= r.e) mid = r.b + (r.e - r.b) / 2;  // (not reached: every inner node has its split)
    stack.push_back({mid, r.e, r.depth + 1});
    stack.push_back({r.b, mid, r.depth + 1});
  }
  for (size_t k = 0; k < G.cell0.size(); ++k) {
    const int64_t e = k + 1 < G.cell0.size() ? G.cell0[k + 1] : nc;
    for (int64_t s = G.cell0[k]; s < e; ++s) G.of_cell[s] = (int32_t)k;
  }
  G.cell0.push_back((int32_t)nc);
  G.ng = (int64_t)G.cell0.size() - 1;
  const int64_t ng = G.ng;
  // origins: mean of member centroids rounded to a multiple of 2^-15
  G.orig.assign(3 * ng, 0.0);
  for (int64_t a = 0; a < ng; ++a) {
    double s[3] = {0, 0, 0};
    for (int32_t sc = G.cell0[a]; sc < G.cell0[a + 1]; ++sc)
      for (int q = 0; q < 3; ++q) s[q] += g.ccen[3 * (int64_t)order[sc] + q];
    double n = G.cell0[a + 1] - G.cell0[a];
    for (int q = 0; q < 3; ++q) G.orig[3 * a + q] = std::ldexp(std::nearbyint(std::ldexp(s[q] / n, 15)), -15);
  }
  // group pairs: every cell pair maps to (group(sc), group(sd), img) with group(sc) <= group(sd)
  // since groups are consecutive ranges of the sorted order; (A, A, 0) is the self entry.
  std::vector<int64_t> pstart(ng + 1, 0);
  {
    int64_t p = 0;
    for (int64_t a = 0; a < ng; ++a) {
      pstart[a] = p;
      while (p < (int64_t)pairs.size() && pairs[p].sc < G.cell0[a + 1]) ++p;
    }
    pstart[ng] = (int64_t)pairs.size();
  }
  std::vector<std::vector<int64_t>> lists(ng);  // key = B * 32 + code
  parallel_for(ng, [&](int64_t b, int64_t e, int) {
    for (int64_t a = b; a < e; ++a) {
      std::vector<int64_t> &L = lists[a];
      L.push_back(a * 32 + 13);
      for (int64_t p = pstart[a]; p < pstart[a + 1]; ++p) {
        const CellPair &cp = pairs[p];
        int64_t B = G.of_cell[cp.sd];
        int code = img_code(cp.img[0], cp.img[1], cp.img[2]);
        if (B == a && code == 13) continue;
        if (B == a && code < 13) code = 26 - code;
        L.push_back(B * 32 + code);
      }
      std::sort(L.begin(), L.end());
      L.erase(std::unique(L.begin(), L.end()), L.end());
    }
  });
  G.e_off.assign(ng + 1, 0);
  for (int64_t a = 0; a < ng; ++a) G.e_off[a + 1] = G.e_off[a] + (int64_t)lists[a].size();
  const int64_t E = G.e_off[ng];
  G.e_B.assign(E, 0);
  G.e_img.assign(3 * E, 0);
  std::vector<int64_t> rcnt(ng + 1, 0);
  for (int64_t a = 0; a < ng; ++a) {
    int64_t e = G.e_off[a];
    for (int64_t key : lists[a]) {
      int32_t B = (int32_t)(key / 32);
      int code = (int)(key % 32);
      G.e_B[e] = B;
      G.e_img[3 * e] = (int8_t)(code / 9 - 1);
      G.e_img[3 * e + 1] = (int8_t)((code / 3) % 3 - 1);
      G.e_img[3 * e + 2] = (int8_t)(code % 3 - 1);
      rcnt[B + 1]++;
      ++e;
    }
    std::vector<int64_t>().swap(lists[a]);
  }
  for (int64_t b = 0; b < ng; ++b) rcnt[b + 1] += rcnt[b];
  G.r_off = rcnt;
  G.r_e.assign(E, 0);
  std::vector<int64_t> fill(G.r_off.begin(), G.r_off.end() - 1);
  for (int64_t e = 0; e < E; ++e) G.r_e[fill[G.e_B[e]]++] = (int32_t)e;

  // needed j-cells of every non-self entry.  A cell pair (sc, sd, img), sc <= sd, is the physical
  // pair {cell sc, cell sd + img}; in group terms it is evaluated by entry (A, B, img) with j in sd,
  // or, for A == B and a negative image, by entry (A, A, -img) with j in sc.
  std::vector<std::vector<int64_t>> nlists(ng);  // key = entry * 2^31 + j-cell
  parallel_for(ng, [&](int64_t b, int64_t e, int) {
    for (int64_t a = b; a < e; ++a) {
      std::vector<int64_t> &L = nlists[a];
      const int64_t eb = G.e_off[a], ee = G.e_off[a + 1];
      auto find_entry = [&](int32_t B, int code) -> int64_t {
        // entries of A are sorted by (B, code)
        int64_t lo = eb, hi = ee;
        const int64_t key = (int64_t)B * 32 + code;
        while (lo < hi) {
          const int64_t mid = (lo + hi) / 2;
          const int64_t k = (int64_t)G.e_B[mid] * 32 +
                            (9 * (G.e_img[3 * mid] + 1) + 3 * (G.e_img[3 * mid + 1] + 1) + (G.e_img[3 * mid + 2] + 1));
          if (k < key) lo = mid + 1; else hi = mid;
        }
        return lo;
      };
      for (int64_t p = pstart[a]; p < pstart[a + 1]; ++p) {
        const CellPair &cp = pairs[p];
        const int32_t B = G.of_cell[cp.sd];
        int code = img_code(cp.img[0], cp.img[1], cp.img[2]);
        int32_t jcell = cp.sd;
        if (B == a && code == 13) continue;  // inside the self entry
        if (B == a && code < 13) {
          code = 26 - code;
          jcell = cp.sc;
        }
        const int64_t en = find_entry(B, code);
        L.push_back(en * (1LL << 31) + jcell);
      }
      std::sort(L.begin(), L.end());
      L.erase(std::unique(L.begin(), L.end()), L.end());
    }
  });
  G.nl_off.assign(ng + 1, 0);
  for (int64_t a = 0; a < ng; ++a) G.nl_off[a + 1] = G.nl_off[a] + (int64_t)nlists[a].size();
  const int64_t NL = G.nl_off[ng];
  G.nl_e.assign(NL, 0);
  G.nl_d.assign(NL, 0);
  G.rc_off.assign(nc + 1, 0);
  for (int64_t a = 0; a < ng; ++a) {
    int64_t k = G.nl_off[a];
    for (int64_t key : nlists[a]) {
      G.nl_e[k] = (int32_t)(key >> 31);
      G.nl_d[k] = (int32_t)(key & ((1LL << 31) - 1));
      G.rc_off[G.nl_d[k] + 1]++;
      ++k;
    }
    std::vector<int64_t>().swap(nlists[a]);
  }
  for (int64_t c = 0; c < nc; ++c) G.rc_off[c + 1] += G.rc_off[c];
  G.rc_e.assign(NL, 0);
  G.nl_r.assign(NL, 0);
  std::vector<int64_t> cfill(G.rc_off.begin(), G.rc_off.end() - 1);
  for (int64_t k = 0; k < NL; ++k) {
    const int32_t d = G.nl_d[k];
    G.nl_r[k] = (int32_t)(1 + cfill[d] - G.rc_off[d]);
    G.rc_e[cfill[d]++] = G.nl_e[k];
  }
  return AICA_OK;
}

}  // namespace aica
