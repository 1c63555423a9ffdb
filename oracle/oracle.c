/*
 * FP64 CPU oracle for the AICA Lennard-Jones hot path (test infrastructure).
 *
 * This file is test infrastructure only: the tests, the smoke check and the
 * CPU-baseline leg of the benchmark call it.  It shares no code with the HIP
 * library and computes every result from its plain definition:
 *
 *   - Lennard-Jones pair terms with a hard cut-off (Sec. 2.2: potentials are
 *     set to zero beyond r_cut), Lorentz-Berthelot mixing for mixtures;
 *   - forces, potential energy, virial and pair count by all-pairs summation
 *     over explicit periodic images (Fig. "periodic boundaries": the minimum
 *     image is the serial special case of referred molecules);
 *   - the interacting cell pairs (direct interaction lists, Sec. 2.2 and
 *     App. A.1, with the closest-point predicate and guard distance of
 *     Sec. 2.2) by brute force over every cell pair and lattice image;
 *   - point location by testing every cell;
 *   - the analytic adjoint of L = sum_i G_i . F_i + gamma * U.
 *
 * No blocking, fusion or reordering beyond the definitions is used, except
 * two obviously valid shortcuts in the brute-force cell distance test: a
 * vertex pair closer than the threshold proves the cells are in range, and
 * axis-aligned bounding boxes farther apart than the threshold prove they are
 * not.  Row sums use a fixed order, so results are bit-reproducible.
 *
 * Images: for each periodic lattice vector v_k the oracle sums n_k in
 * [-m_k, m_k] with m_k = ceil(rc / |v_k|) (lattice vectors must be mutually
 * orthogonal).  When rc < |v_k|/2 this reduces to the minimum image.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OC_OK 0
#define OC_E_INVAL -1
#define OC_E_MESH -2

/* ------------------------------------------------------------------ LJ pair terms */

/* Lorentz-Berthelot mixing: sigma_ab = (sigma_a+sigma_b)/2, eps_ab = sqrt(eps_a eps_b). */
static void oc_mix(const double *eps, const double *sig, int a, int b, double *e, double *s) {
  *e = (a == b) ? eps[a] : sqrt(eps[a] * eps[b]);
  *s = (a == b) ? sig[a] : 0.5 * (sig[a] + sig[b]);
}

/* u(r) = 4 eps [(sig/r)^12 - (sig/r)^6];  g(s) with F_ab = g * d, s = |d|^2:
 * g = 24 eps [2 sig^12 s^-7 - sig^6 s^-4]. */
void oc_lj(double s, double eps, double sig, double *u, double *g) {
  double sr2 = sig * sig / s;
  double sr6 = sr2 * sr2 * sr2;
  double sr12 = sr6 * sr6;
  *u = 4.0 * eps * (sr12 - sr6);
  *g = 24.0 * eps * (2.0 * sr12 - sr6) / s;
}

/* ------------------------------------------------------------------ images */

static int oc_images(int nper, const double *lat, double rc, double *img /*[max][3]*/, int *code /*[max][3]*/, int maxn) {
  int m[3] = {0, 0, 0};
  for (int k = 0; k < nper; ++k) {
    double len = sqrt(lat[3 * k] * lat[3 * k] + lat[3 * k + 1] * lat[3 * k + 1] + lat[3 * k + 2] * lat[3 * k + 2]);
    if (!(len > 0)) return -1;
    m[k] = (int)ceil(rc / len);
    for (int l = 0; l < k; ++l) {
      double dot = lat[3 * k] * lat[3 * l] + lat[3 * k + 1] * lat[3 * l + 1] + lat[3 * k + 2] * lat[3 * l + 2];
      if (fabs(dot) > 1e-12 * len * len) return -1; /* orthogonal lattices only */
    }
  }
  int cnt = 0;
  for (int a = -m[0]; a <= m[0]; ++a)
    for (int b = -m[1]; b <= m[1]; ++b)
      for (int c = -m[2]; c <= m[2]; ++c) {
        int n[3] = {a, b, c};
        if (cnt >= maxn) return -1;
        for (int q = 0; q < 3; ++q) {
          img[3 * cnt + q] = 0.0;
          code[3 * cnt + q] = n[q];
        }
        for (int k = 0; k < nper; ++k)
          for (int q = 0; q < 3; ++q) img[3 * cnt + q] += n[k] * lat[3 * k + q];
        ++cnt;
      }
  return cnt;
}

#define OC_MAXIMG 4096

/* ------------------------------------------------------------------ forces, energy, virial */

/* Row a collects sum over b, n with (b,n) != (a,0) and s < rc^2 of F_ab; U and W
 * collect half of each term per row (every pair is seen from both rows). */
static void oc_row(int64_t a, int64_t n, const double *x, const int32_t *sp, const double *eps, const double *sig,
                   double rc2, int nimg, const double *img, double *Fa, double *Ua, double *Wa, int64_t *npa) {
  double f0 = 0, f1 = 0, f2 = 0, u2 = 0, w2 = 0;
  int64_t cnt = 0;
  for (int64_t b = 0; b < n; ++b) {
    double e, sg;
    oc_mix(eps, sig, sp[a], sp[b], &e, &sg);
    for (int k = 0; k < nimg; ++k) {
      if (b == a && img[3 * k] == 0 && img[3 * k + 1] == 0 && img[3 * k + 2] == 0) continue;
      double d0 = x[3 * a] - (x[3 * b] + img[3 * k]);
      double d1 = x[3 * a + 1] - (x[3 * b + 1] + img[3 * k + 1]);
      double d2 = x[3 * a + 2] - (x[3 * b + 2] + img[3 * k + 2]);
      double s = d0 * d0 + d1 * d1 + d2 * d2;
      if (s < rc2) {
        double u, g;
        oc_lj(s, e, sg, &u, &g);
        f0 += g * d0;
        f1 += g * d1;
        f2 += g * d2;
        u2 += 0.5 * u;
        w2 += 0.5 * g * s;
        ++cnt;
      }
    }
  }
  Fa[0] = f0;
  Fa[1] = f1;
  Fa[2] = f2;
  *Ua = u2;
  *Wa = w2;
  *npa = cnt;
}

int oc_forces(int64_t n, const double *x, const int32_t *sp, int32_t nsp, const double *eps, const double *sig,
              double rc, int32_t nper, const double *lat, double *F, double *U, double *W, int64_t *npairs) {
  static double img[3 * OC_MAXIMG];
  static int code[3 * OC_MAXIMG];
  int nimg = oc_images(nper, lat, rc, img, code, OC_MAXIMG);
  if (nimg < 0 || n < 0 || nsp < 1) return OC_E_INVAL;
  double *Ur = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
  double *Wr = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
  int64_t *Cr = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
  double rc2 = rc * rc;
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < n; ++a) oc_row(a, n, x, sp, eps, sig, rc2, nimg, img, F + 3 * a, Ur + a, Wr + a, Cr + a);
  double u = 0, w = 0;
  int64_t c = 0;
  for (int64_t a = 0; a < n; ++a) {
    u += Ur[a];
    w += Wr[a];
    c += Cr[a];
  }
  *U = u;
  *W = w;
  *npairs = c / 2;
  free(Ur);
  free(Wr);
  free(Cr);
  return OC_OK;
}

/* Forces on selected rows only (each against all n molecules): the sampled
 * check for workloads too large for all pairs.  Urow/Wrow/cnt are per-row half sums. */
int oc_forces_rows(int64_t n, const double *x, const int32_t *sp, int32_t nsp, const double *eps, const double *sig,
                   double rc, int32_t nper, const double *lat, int64_t nrows, const int64_t *rows, double *F,
                   double *Urow, double *Wrow, int64_t *cnt) {
  static double img[3 * OC_MAXIMG];
  static int code[3 * OC_MAXIMG];
  int nimg = oc_images(nper, lat, rc, img, code, OC_MAXIMG);
  if (nimg < 0 || nsp < 1) return OC_E_INVAL;
  double rc2 = rc * rc;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < nrows; ++r) oc_row(rows[r], n, x, sp, eps, sig, rc2, nimg, img, F + 3 * r, Urow + r, Wrow + r, cnt + r);
  return OC_OK;
}

/* Pair set: every unordered pair {a, b+image} with s < rc^2, reported as
 * (a, b, n) with a < b and d = x_a - x_b - sum_k n_k v_k.  Returns the count;
 * arrays may be NULL to count only. */
int64_t oc_pairs(int64_t n, const double *x, double rc, int32_t nper, const double *lat, int64_t cap, int32_t *pa,
                 int32_t *pb, int8_t *pn) {
  static double img[3 * OC_MAXIMG];
  static int code[3 * OC_MAXIMG];
  int nimg = oc_images(nper, lat, rc, img, code, OC_MAXIMG);
  if (nimg < 0) return -1;
  double rc2 = rc * rc;
  int64_t cnt = 0;
  for (int64_t a = 0; a < n; ++a)
    for (int64_t b = a + 1; b < n; ++b)
      for (int k = 0; k < nimg; ++k) {
        double d0 = x[3 * a] - (x[3 * b] + img[3 * k]);
        double d1 = x[3 * a + 1] - (x[3 * b + 1] + img[3 * k + 1]);
        double d2 = x[3 * a + 2] - (x[3 * b + 2] + img[3 * k + 2]);
        double s = d0 * d0 + d1 * d1 + d2 * d2;
        if (s < rc2) {
          if (pa && cnt < cap) {
            pa[cnt] = (int32_t)a;
            pb[cnt] = (int32_t)b;
            pn[3 * cnt] = (int8_t)code[3 * k];
            pn[3 * cnt + 1] = (int8_t)code[3 * k + 1];
            pn[3 * cnt + 2] = (int8_t)code[3 * k + 2];
          }
          ++cnt;
        }
      }
  return cnt;
}

/* ------------------------------------------------------------------ adjoint */

/* L = sum_i G_i . F_i + gamma U.  Per pair (a,b,image) with d = x_a - x_b', s = d.d:
 *   l = (G_a - G_b).d g(s) + gamma u(s)
 *   dl/dd = g (G_a-G_b) + [2 g'(s) ((G_a-G_b).d) - gamma g] d      (du/ds = -g/2)
 *   dl/deps_ab = l / eps_ab
 *   dl/dsig_ab = ((G_a-G_b).d) dg/dsig + gamma du/dsig
 * with g' = dg/ds = 24 eps (-14 sig^12 s^-8 + 4 sig^6 s^-5),
 *      dg/dsig = (24 eps/sig)(24 sig^12 s^-7 - 6 sig^6 s^-4),
 *      du/dsig = (24 eps/sig)(2 sig^12 s^-6 - sig^6 s^-3).
 * Lorentz-Berthelot chain rule to per-species parameters:
 *   d eps_ab/d eps_a = eps_ab/(2 eps_a) (a != b), 1 (a == b);
 *   d sig_ab/d sig_a = 1/2 (a != b), 1 (a == b).
 * The cut-off radius is absolute, so sigma does not move it.
 * Row a collects dL/dx_a = sum_b dl/dd(a,b) (each pair seen from both rows, with
 * dl/dd symmetric under a<->b, d -> -d); parameter sums take half per row. */
int oc_adjoint(int64_t n, const double *x, const int32_t *sp, int32_t nsp, const double *eps, const double *sig,
               double rc, int32_t nper, const double *lat, const double *G, double gamma, double *gx, double *geps,
               double *gsig, double *L) {
  static double img[3 * OC_MAXIMG];
  static int code[3 * OC_MAXIMG];
  int nimg = oc_images(nper, lat, rc, img, code, OC_MAXIMG);
  if (nimg < 0 || nsp < 1 || nsp > 8) return OC_E_INVAL;
  double rc2 = rc * rc;
  /* per-row partial sums for the species-pair parameter gradients and L */
  double *pe = (double *)calloc((size_t)(n > 0 ? n : 1) * 64, sizeof(double));
  double *ps = (double *)calloc((size_t)(n > 0 ? n : 1) * 64, sizeof(double));
  double *pl = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < n; ++a) {
    double v0 = 0, v1 = 0, v2 = 0, la = 0;
    for (int64_t b = 0; b < n; ++b) {
      double e, sg;
      oc_mix(eps, sig, sp[a], sp[b], &e, &sg);
      double dg0 = G[3 * a] - G[3 * b], dg1 = G[3 * a + 1] - G[3 * b + 1], dg2 = G[3 * a + 2] - G[3 * b + 2];
      for (int k = 0; k < nimg; ++k) {
        if (b == a && img[3 * k] == 0 && img[3 * k + 1] == 0 && img[3 * k + 2] == 0) continue;
        double d0 = x[3 * a] - (x[3 * b] + img[3 * k]);
        double d1 = x[3 * a + 1] - (x[3 * b + 1] + img[3 * k + 1]);
        double d2 = x[3 * a + 2] - (x[3 * b + 2] + img[3 * k + 2]);
        double s = d0 * d0 + d1 * d1 + d2 * d2;
        if (!(s < rc2)) continue;
        double sr2 = sg * sg / s, sr6 = sr2 * sr2 * sr2, sr12 = sr6 * sr6;
        double u = 4.0 * e * (sr12 - sr6);
        double g = 24.0 * e * (2.0 * sr12 - sr6) / s;
        double gp = 24.0 * e * (-14.0 * sr12 + 4.0 * sr6) / (s * s);
        double gd = dg0 * d0 + dg1 * d1 + dg2 * d2;
        double c = 2.0 * gp * gd - gamma * g;
        v0 += g * dg0 + c * d0;
        v1 += g * dg1 + c * d1;
        v2 += g * dg2 + c * d2;
        double l = gd * g + gamma * u;
        la += 0.5 * l;
        double dgds = (24.0 * e / sg) * (24.0 * sr12 - 6.0 * sr6) / s;
        double duds = (24.0 * e / sg) * (2.0 * sr12 - sr6);
        int t = sp[a] * 8 + sp[b];
        pe[64 * a + t] += 0.5 * l / e;
        ps[64 * a + t] += 0.5 * (gd * dgds + gamma * duds);
      }
    }
    gx[3 * a] = v0;
    gx[3 * a + 1] = v1;
    gx[3 * a + 2] = v2;
    pl[a] = la;
  }
  double se[64], ss[64];
  memset(se, 0, sizeof se);
  memset(ss, 0, sizeof ss);
  double lsum = 0;
  for (int64_t a = 0; a < n; ++a) {
    for (int t = 0; t < 64; ++t) {
      se[t] += pe[64 * a + t];
      ss[t] += ps[64 * a + t];
    }
    lsum += pl[a];
  }
  for (int p = 0; p < nsp; ++p) {
    geps[p] = 0;
    gsig[p] = 0;
  }
  for (int a = 0; a < nsp; ++a)
    for (int b = 0; b < nsp; ++b) {
      int t = a * 8 + b;
      double e, sg;
      oc_mix(eps, sig, a, b, &e, &sg);
      if (a == b) {
        geps[a] += se[t];
        gsig[a] += ss[t];
      } else {
        /* ordered (a,b) and (b,a) each carry half of the unordered pair's share */
        geps[a] += se[t] * e / (2.0 * eps[a]);
        geps[b] += se[t] * e / (2.0 * eps[b]);
        gsig[a] += 0.5 * ss[t];
        gsig[b] += 0.5 * ss[t];
      }
    }
  if (L) *L = lsum;
  free(pe);
  free(ps);
  free(pl);
  return OC_OK;
}

/* ------------------------------------------------------------------ mesh geometry */

typedef struct {
  int64_t n_points;
  const double *points;
  int64_t n_faces;
  const int64_t *face_off;
  const int32_t *face_pts;
  const int32_t *owner;
  const int32_t *neighbour;
  int64_t n_cells;
} oc_mesh;

/* Boundary triangles of one cell: every face of the cell is fanned around the
 * mean of its vertices, oriented out of the cell.  tri[9*k..] holds 3 points. */
typedef struct {
  int ntri;
  double *tri;       /* [ntri][3][3] */
  double cen[3];     /* vertex mean of the cell's distinct vertices */
  double lo[3], hi[3];
  int nv;
  double *v;         /* distinct vertices [nv][3] */
} oc_cell;

static int oc_build_cells(const oc_mesh *m, oc_cell **out) {
  int64_t nc = m->n_cells;
  oc_cell *cells = (oc_cell *)calloc((size_t)nc, sizeof(oc_cell));
  int *ntri = (int *)calloc((size_t)nc, sizeof(int));
  for (int64_t f = 0; f < m->n_faces; ++f) {
    int64_t len = m->face_off[f + 1] - m->face_off[f];
    if (len < 3) {
      free(cells);
      free(ntri);
      return OC_E_MESH;
    }
    if (m->owner[f] < 0 || m->owner[f] >= nc) {
      free(cells);
      free(ntri);
      return OC_E_MESH;
    }
    ntri[m->owner[f]] += (int)len;
    if (m->neighbour[f] >= 0) ntri[m->neighbour[f]] += (int)len;
  }
  for (int64_t c = 0; c < nc; ++c) {
    cells[c].tri = (double *)malloc(sizeof(double) * 9 * (ntri[c] > 0 ? ntri[c] : 1));
    cells[c].v = (double *)malloc(sizeof(double) * 3 * (ntri[c] > 0 ? ntri[c] : 1));
  }
  /* distinct vertex lists */
  int32_t **vid = (int32_t **)calloc((size_t)nc, sizeof(int32_t *));
  for (int64_t c = 0; c < nc; ++c) vid[c] = (int32_t *)malloc(sizeof(int32_t) * (ntri[c] > 0 ? ntri[c] : 1));
  for (int64_t f = 0; f < m->n_faces; ++f) {
    int64_t b = m->face_off[f], len = m->face_off[f + 1] - b;
    double fc[3] = {0, 0, 0};
    for (int64_t k = 0; k < len; ++k)
      for (int q = 0; q < 3; ++q) fc[q] += m->points[3 * (int64_t)m->face_pts[b + k] + q];
    for (int q = 0; q < 3; ++q) fc[q] /= (double)len;
    for (int side = 0; side < 2; ++side) {
      int32_t c = side == 0 ? m->owner[f] : m->neighbour[f];
      if (c < 0) continue;
      oc_cell *C = &cells[c];
      for (int64_t k = 0; k < len; ++k) {
        int64_t ia = m->face_pts[b + k], ib = m->face_pts[b + (k + 1) % len];
        if (side == 1) {
          int64_t t = ia;
          ia = ib;
          ib = t;
        }
        double *T = C->tri + 9 * C->ntri;
        for (int q = 0; q < 3; ++q) {
          T[q] = fc[q];
          T[3 + q] = m->points[3 * ia + q];
          T[6 + q] = m->points[3 * ib + q];
        }
        C->ntri++;
        int32_t pv = m->face_pts[b + k];
        int seen = 0;
        for (int j = 0; j < C->nv; ++j)
          if (vid[c][j] == pv) seen = 1;
        if (!seen) {
          vid[c][C->nv] = pv;
          for (int q = 0; q < 3; ++q) C->v[3 * C->nv + q] = m->points[3 * (int64_t)pv + q];
          C->nv++;
        }
      }
    }
  }
  for (int64_t c = 0; c < nc; ++c) {
    oc_cell *C = &cells[c];
    for (int q = 0; q < 3; ++q) {
      C->cen[q] = 0;
      C->lo[q] = 1e300;
      C->hi[q] = -1e300;
    }
    for (int j = 0; j < C->nv; ++j)
      for (int q = 0; q < 3; ++q) {
        C->cen[q] += C->v[3 * j + q];
        if (C->v[3 * j + q] < C->lo[q]) C->lo[q] = C->v[3 * j + q];
        if (C->v[3 * j + q] > C->hi[q]) C->hi[q] = C->v[3 * j + q];
      }
    for (int q = 0; q < 3; ++q) C->cen[q] /= (C->nv > 0 ? C->nv : 1);
    free(vid[c]);
  }
  free(vid);
  free(ntri);
  *out = cells;
  return OC_OK;
}

static void oc_free_cells(oc_cell *cells, int64_t nc) {
  for (int64_t c = 0; c < nc; ++c) {
    free(cells[c].tri);
    free(cells[c].v);
  }
  free(cells);
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void sub3(const double *a, const double *b, double *o) {
  o[0] = a[0] - b[0];
  o[1] = a[1] - b[1];
  o[2] = a[2] - b[2];
}
static void cross3(const double *a, const double *b, double *o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

/* orientation (b-a).((c-a)x(d-a)) */
static double orient(const double *a, const double *b, const double *c, const double *d) {
  double u[3], v[3], w[3], x[3];
  sub3(b, a, u);
  sub3(c, a, v);
  sub3(d, a, w);
  cross3(v, w, x);
  return dot3(u, x);
}

/* squared distance from p to segment [a,b] */
static double pt_seg2(const double *p, const double *a, const double *b) {
  double ab[3], ap[3];
  sub3(b, a, ab);
  sub3(p, a, ap);
  double L = dot3(ab, ab);
  double t = L > 0 ? dot3(ap, ab) / L : 0.0;
  if (t < 0) t = 0;
  if (t > 1) t = 1;
  double c[3] = {a[0] + t * ab[0] - p[0], a[1] + t * ab[1] - p[1], a[2] + t * ab[2] - p[2]};
  return dot3(c, c);
}

/* squared distance from p to triangle (a,b,c): the plane foot point if it lies
 * inside the triangle (all barycentric weights >= 0), else the nearest edge. */
static double pt_tri2(const double *p, const double *a, const double *b, const double *c) {
  double ab[3], ac[3], n[3], ap[3];
  sub3(b, a, ab);
  sub3(c, a, ac);
  cross3(ab, ac, n);
  double nn = dot3(n, n);
  double best = pt_seg2(p, a, b);
  double t = pt_seg2(p, b, c);
  if (t < best) best = t;
  t = pt_seg2(p, c, a);
  if (t < best) best = t;
  if (nn > 0) {
    sub3(p, a, ap);
    double h = dot3(ap, n) / nn;
    double f[3] = {p[0] - h * n[0], p[1] - h * n[1], p[2] - h * n[2]};
    /* barycentric weights of f via sub-triangle areas along n */
    double e0[3], e1[3], x[3];
    double fa[3], fb[3], fc[3];
    sub3(a, f, fa);
    sub3(b, f, fb);
    sub3(c, f, fc);
    cross3(fb, fc, x);
    double wa = dot3(x, n);
    cross3(fc, fa, x);
    double wb = dot3(x, n);
    cross3(fa, fb, x);
    double wc = dot3(x, n);
    (void)e0;
    (void)e1;
    if (wa >= 0 && wb >= 0 && wc >= 0) {
      double d = h * h * nn;
      if (d < best) best = d;
    }
  }
  return best;
}

/* squared distance between segments [p0,p1] and [q0,q1]: the minimum of the
 * convex quadratic over the unit square is at the interior stationary point
 * (when it exists and lies inside) or on one of the four sides. */
static double seg_seg2(const double *p0, const double *p1, const double *q0, const double *q1) {
  double best = pt_seg2(p0, q0, q1), t;
  t = pt_seg2(p1, q0, q1);
  if (t < best) best = t;
  t = pt_seg2(q0, p0, p1);
  if (t < best) best = t;
  t = pt_seg2(q1, p0, p1);
  if (t < best) best = t;
  double d1[3], d2[3], r[3];
  sub3(p1, p0, d1);
  sub3(q1, q0, d2);
  sub3(p0, q0, r);
  double a = dot3(d1, d1), e = dot3(d2, d2), b = dot3(d1, d2), c = dot3(d1, r), f = dot3(d2, r);
  double den = a * e - b * b;
  if (den > 1e-300 * (a * e > 0 ? a * e : 1)) {
    double s = (b * f - c * e) / den;
    double u = (a * f - b * c) / den;
    if (s > 0 && s < 1 && u > 0 && u < 1) {
      double w[3] = {p0[0] + s * d1[0] - q0[0] - u * d2[0], p0[1] + s * d1[1] - q0[1] - u * d2[1],
                     p0[2] + s * d1[2] - q0[2] - u * d2[2]};
      t = dot3(w, w);
      if (t < best) best = t;
    }
  }
  return best;
}

/* squared distance between triangles that do not interpenetrate */
static double tri_tri2(const double *A, const double *B) {
  double best = 1e300, t;
  for (int i = 0; i < 3; ++i) {
    t = pt_tri2(A + 3 * i, B, B + 3, B + 6);
    if (t < best) best = t;
    t = pt_tri2(B + 3 * i, A, A + 3, A + 6);
    if (t < best) best = t;
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      t = seg_seg2(A + 3 * i, A + 3 * ((i + 1) % 3), B + 3 * j, B + 3 * ((j + 1) % 3));
      if (t < best) best = t;
    }
  return best;
}

/* Is the closest distance between cell c and cell d translated by T below R? */
static int oc_cells_in_range(const oc_cell *C, const oc_cell *D, const double *T, double R) {
  double R2 = R * R;
  /* bounding boxes farther apart than R: not in range */
  double g2 = 0;
  for (int q = 0; q < 3; ++q) {
    double lo = D->lo[q] + T[q], hi = D->hi[q] + T[q];
    double gap = 0;
    if (lo > C->hi[q]) gap = lo - C->hi[q];
    if (C->lo[q] > hi) gap = C->lo[q] - hi;
    g2 += gap * gap;
  }
  if (g2 >= R2) return 0;
  /* a vertex pair closer than R: in range */
  for (int i = 0; i < C->nv; ++i)
    for (int j = 0; j < D->nv; ++j) {
      double d[3] = {C->v[3 * i] - D->v[3 * j] - T[0], C->v[3 * i + 1] - D->v[3 * j + 1] - T[1],
                     C->v[3 * i + 2] - D->v[3 * j + 2] - T[2]};
      if (dot3(d, d) < R2) return 1;
    }
  /* full minimum over boundary triangle pairs */
  double Bt[9];
  for (int i = 0; i < C->ntri; ++i)
    for (int j = 0; j < D->ntri; ++j) {
      for (int k = 0; k < 3; ++k)
        for (int q = 0; q < 3; ++q) Bt[3 * k + q] = D->tri[9 * j + 3 * k + q] + T[q];
      if (tri_tri2(C->tri + 9 * i, Bt) < R2) return 1;
    }
  return 0;
}

static int oc_mesh_from(int64_t n_points, const double *points, int64_t n_faces, const int64_t *face_off,
                        const int32_t *face_pts, const int32_t *owner, const int32_t *neighbour, int64_t n_cells,
                        oc_mesh *m) {
  m->n_points = n_points;
  m->points = points;
  m->n_faces = n_faces;
  m->face_off = face_off;
  m->face_pts = face_pts;
  m->owner = owner;
  m->neighbour = neighbour;
  m->n_cells = n_cells;
  return OC_OK;
}

/* Exact closest distance between cell c and cell d shifted by T (for pins). */
double oc_cell_distance(int64_t n_points, const double *points, int64_t n_faces, const int64_t *face_off,
                        const int32_t *face_pts, const int32_t *owner, const int32_t *neighbour, int64_t n_cells,
                        int32_t c, int32_t d, const double *T) {
  oc_mesh m;
  oc_mesh_from(n_points, points, n_faces, face_off, face_pts, owner, neighbour, n_cells, &m);
  oc_cell *cells;
  if (oc_build_cells(&m, &cells) != OC_OK) return -1;
  double best = 1e300, Bt[9];
  oc_cell *C = &cells[c], *D = &cells[d];
  for (int i = 0; i < C->ntri; ++i)
    for (int j = 0; j < D->ntri; ++j) {
      for (int k = 0; k < 3; ++k)
        for (int q = 0; q < 3; ++q) Bt[3 * k + q] = D->tri[9 * j + 3 * k + q] + T[q];
      double t = tri_tri2(C->tri + 9 * i, Bt);
      if (t < best) best = t;
    }
  oc_free_cells(cells, n_cells);
  return sqrt(best);
}

/* Brute-force interacting cell pairs: every (c, d, n) with closest distance
 * between cell c and cell d + sum_k n_k v_k below rc + guard, n_k in {-1,0,1},
 * reported once: c < d, or c == d with n lexicographically positive.  Returns
 * the count (arrays may be NULL to count only), or <0 on error. */
/* The paper's own cell-pair predicate (Sec. 2.2, App. A.1): some vertex of c and some vertex of d + T
 * are closer than R.  Brute force over all vertex pairs. */
static int oc_vertices_in_range(const oc_cell *c, const oc_cell *d, const double *T, double R) {
  for (int i = 0; i < c->nv; ++i)
    for (int j = 0; j < d->nv; ++j) {
      double s = 0;
      for (int q = 0; q < 3; ++q) {
        double e = c->v[3 * i + q] - (d->v[3 * j + q] + T[q]);
        s += e * e;
      }
      if (s < R * R) return 1;
    }
  return 0;
}

/* Interacting cell pairs, canonical (c < d, or c == d with the lattice image lexicographically
 * positive).  predicate 0: closest distance between the closed cells below rc + guard; 1: the paper's
 * vertex-to-vertex distance below rc + guard. */
int64_t oc_dil(int64_t n_points, const double *points, int64_t n_faces, const int64_t *face_off,
               const int32_t *face_pts, const int32_t *owner, const int32_t *neighbour, int64_t n_cells,
               int32_t nper, const double *lat, double rc, double guard, int32_t predicate, int64_t cap, int32_t *oc,
               int32_t *od, int8_t *on) {
  oc_mesh m;
  oc_mesh_from(n_points, points, n_faces, face_off, face_pts, owner, neighbour, n_cells, &m);
  oc_cell *cells;
  if (oc_build_cells(&m, &cells) != OC_OK) return OC_E_MESH;
  double R = rc + guard;
  int nimg = 1;
  for (int k = 0; k < nper; ++k) nimg *= 3;
  int64_t cnt = 0;
  for (int64_t c = 0; c < n_cells; ++c)
    for (int64_t d = c; d < n_cells; ++d)
      for (int im = 0; im < nimg; ++im) {
        int n[3] = {0, 0, 0}, r = im;
        for (int k = 0; k < nper; ++k) {
          n[k] = r % 3 - 1;
          r /= 3;
        }
        if (c == d) {
          /* keep n lexicographically > 0 only (n = 0 is the cell itself) */
          int pos = 0;
          for (int k = 0; k < 3; ++k) {
            if (n[k] > 0) {
              pos = 1;
              break;
            }
            if (n[k] < 0) break;
          }
          if (!pos) continue;
        }
        double T[3] = {0, 0, 0};
        for (int k = 0; k < nper; ++k)
          for (int q = 0; q < 3; ++q) T[q] += n[k] * lat[3 * k + q];
        if (predicate == 1 ? oc_vertices_in_range(&cells[c], &cells[d], T, R)
                           : oc_cells_in_range(&cells[c], &cells[d], T, R)) {
          if (oc && cnt < cap) {
            oc[cnt] = (int32_t)c;
            od[cnt] = (int32_t)d;
            for (int k = 0; k < 3; ++k) on[3 * cnt + k] = (int8_t)n[k];
          }
          ++cnt;
        }
      }
  oc_free_cells(cells, n_cells);
  return cnt;
}

/* Brute-force point location: the lowest-index cell with some tetrahedron
 * (cell centroid, face centroid, edge) containing the point, with a relative
 * tolerance of 1e-12 of the tetrahedron's volume; -1 if none. */
int oc_locate(int64_t n_points, const double *points, int64_t n_faces, const int64_t *face_off,
              const int32_t *face_pts, const int32_t *owner, const int32_t *neighbour, int64_t n_cells, int64_t n,
              const double *x, int32_t *cell) {
  oc_mesh m;
  oc_mesh_from(n_points, points, n_faces, face_off, face_pts, owner, neighbour, n_cells, &m);
  oc_cell *cells;
  if (oc_build_cells(&m, &cells) != OC_OK) return OC_E_MESH;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const double *p = x + 3 * i;
    int32_t found = -1;
    for (int64_t c = 0; c < n_cells && found < 0; ++c) {
      const oc_cell *C = &cells[c];
      for (int t = 0; t < C->ntri; ++t) {
        const double *a = C->cen, *b = C->tri + 9 * t, *bb = b + 3, *cc = b + 6;
        double v = orient(a, b, bb, cc);
        double tol = -1e-12 * fabs(v);
        if (orient(p, b, bb, cc) >= tol && orient(a, p, bb, cc) >= tol && orient(a, b, p, cc) >= tol &&
            orient(a, b, bb, p) >= tol) {
          found = (int32_t)c;
          break;
        }
      }
    }
    cell[i] = found;
  }
  oc_free_cells(cells, n_cells);
  return OC_OK;
}

/* Smallest tetrahedron volume (cell centroid, face centroid, edge) over the
 * mesh; a valid cell has all of them positive. */
double oc_min_tet_volume(int64_t n_points, const double *points, int64_t n_faces, const int64_t *face_off,
                         const int32_t *face_pts, const int32_t *owner, const int32_t *neighbour, int64_t n_cells) {
  oc_mesh m;
  oc_mesh_from(n_points, points, n_faces, face_off, face_pts, owner, neighbour, n_cells, &m);
  oc_cell *cells;
  if (oc_build_cells(&m, &cells) != OC_OK) return -1e300;
  double best = 1e300;
  for (int64_t c = 0; c < n_cells; ++c)
    for (int t = 0; t < cells[c].ntri; ++t) {
      const double *b = cells[c].tri + 9 * t;
      double v = orient(cells[c].cen, b, b + 3, b + 6) / 6.0;
      if (v < best) best = v;
    }
  oc_free_cells(cells, n_cells);
  return best;
}
