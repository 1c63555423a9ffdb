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
 * Images: every periodic direction k has a referring transform
 * T_k(x) = R_k x + y_k (Sec. 2.2.2, generic form P' = y + R.P).  R_k = I is a
 * lattice translation by y_k; the oracle sums n_k in [-m_k, m_k] with
 * m_k = ceil(rc / |y_k|) (translations must be mutually orthogonal), which is
 * the minimum image when rc < |y_k|/2.  R_k != I (a rotation) must generate a
 * finite group (T_k^K = identity for some K <= 64); the oracle then sums all K
 * distinct powers, so the image sum is complete without any range argument.
 * Image n is the composition T_1^n_1 T_2^n_2 T_3^n_3 (the transforms must
 * commute); rot == NULL means every R_k = I.
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

/* A referring transform x -> R x + y and the powers n of the generators it composes. */
typedef struct {
  double R[9];
  double y[3];
  int n[3];
  int rot; /* 0: R is the identity (a plain translation by y) */
} oc_xf;

static void oc_xf_apply(const oc_xf *t, const double *x, double *o) {
  if (!t->rot) {
    for (int q = 0; q < 3; ++q) o[q] = x[q] + t->y[q];
    return;
  }
  for (int q = 0; q < 3; ++q) o[q] = t->R[3 * q] * x[0] + t->R[3 * q + 1] * x[1] + t->R[3 * q + 2] * x[2] + t->y[q];
}

static void oc_xf_set_rot(oc_xf *t) {
  t->rot = 0;
  for (int i = 0; i < 9; ++i)
    if (t->R[i] != ((i % 4 == 0) ? 1.0 : 0.0)) t->rot = 1;
}

/* rotation part only (how vectors such as forces and G transform) */
static void oc_xf_rotate(const oc_xf *t, const double *v, double *o) {
  for (int q = 0; q < 3; ++q) o[q] = t->R[3 * q] * v[0] + t->R[3 * q + 1] * v[1] + t->R[3 * q + 2] * v[2];
}

/* o = a after b (x -> a(b(x))) */
static void oc_xf_compose(const oc_xf *a, const oc_xf *b, oc_xf *o) {
  oc_xf r;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j)
      r.R[3 * i + j] = a->R[3 * i] * b->R[j] + a->R[3 * i + 1] * b->R[3 + j] + a->R[3 * i + 2] * b->R[6 + j];
    r.y[i] = a->R[3 * i] * b->y[0] + a->R[3 * i + 1] * b->y[1] + a->R[3 * i + 2] * b->y[2] + a->y[i];
  }
  for (int k = 0; k < 3; ++k) r.n[k] = 0;
  oc_xf_set_rot(&r);
  *o = r;
}

static void oc_xf_identity(oc_xf *t) {
  for (int i = 0; i < 9; ++i) t->R[i] = (i % 4 == 0) ? 1.0 : 0.0;
  for (int q = 0; q < 3; ++q) {
    t->y[q] = 0.0;
    t->n[q] = 0;
  }
  t->rot = 0;
}

static int oc_xf_is_identity(const oc_xf *t, double scale) {
  for (int i = 0; i < 9; ++i)
    if (fabs(t->R[i] - ((i % 4 == 0) ? 1.0 : 0.0)) > 1e-12) return 0;
  for (int q = 0; q < 3; ++q)
    if (fabs(t->y[q]) > 1e-9 * scale) return 0;
  return 1;
}

/* Generator k as a transform (rot NULL: the identity rotation). */
static void oc_generator(const double *lat, const double *rot, int k, int inverse, oc_xf *t) {
  oc_xf_identity(t);
  if (rot)
    for (int i = 0; i < 9; ++i) t->R[i] = rot[9 * k + i];
  for (int q = 0; q < 3; ++q) t->y[q] = lat[3 * k + q];
  oc_xf_set_rot(t);
  if (inverse) { /* x = R^T (x' - y) */
    oc_xf v;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) v.R[3 * i + j] = t->R[3 * j + i];
    for (int i = 0; i < 3; ++i) v.y[i] = -(v.R[3 * i] * t->y[0] + v.R[3 * i + 1] * t->y[1] + v.R[3 * i + 2] * t->y[2]);
    for (int q = 0; q < 3; ++q) v.n[q] = 0;
    oc_xf_set_rot(&v);
    *t = v;
  }
}

/* Image sets.  span 0: every image the forces need (translations to ceil(rc/|y|), rotations over their
 * whole finite group); span 1: powers in {-1,0,1} (the cell pairs); span 2: translations to +-2 and
 * rotations over their whole group (used to look for images beyond the first).  Returns the count, or
 * -1 for an invalid set of generators. */
static int oc_transforms(int nper, const double *lat, const double *rot, double rc, int span, oc_xf *out, int maxn) {
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  double scale = 1.0;
  for (int k = 0; k < nper; ++k) scale += fabs(lat[3 * k]) + fabs(lat[3 * k + 1]) + fabs(lat[3 * k + 2]);
  for (int k = 0; k < nper; ++k) {
    oc_xf g;
    oc_generator(lat, rot, k, 0, &g);
    int is_rot = 0;
    for (int i = 0; i < 9; ++i)
      if (g.R[i] != ((i % 4 == 0) ? 1.0 : 0.0)) is_rot = 1;
    if (is_rot) {
      /* orthonormal with determinant +1 */
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double d = g.R[3 * i] * g.R[3 * j] + g.R[3 * i + 1] * g.R[3 * j + 1] + g.R[3 * i + 2] * g.R[3 * j + 2];
          if (fabs(d - (i == j ? 1.0 : 0.0)) > 1e-12) return -1;
        }
      double det = g.R[0] * (g.R[4] * g.R[8] - g.R[5] * g.R[7]) - g.R[1] * (g.R[3] * g.R[8] - g.R[5] * g.R[6]) +
                   g.R[2] * (g.R[3] * g.R[7] - g.R[4] * g.R[6]);
      if (!(det > 0)) return -1;
      oc_xf p = g;
      int K = 1;
      while (!oc_xf_is_identity(&p, scale)) {
        if (++K > 64) return -1; /* not of finite order */
        oc_xf_compose(&g, &p, &p);
      }
      if (span == 1) {
        lo[k] = -1;
        hi[k] = 1;
      } else {
        lo[k] = -((K - 1) / 2);
        hi[k] = K / 2;
      }
    } else {
      double len = sqrt(lat[3 * k] * lat[3 * k] + lat[3 * k + 1] * lat[3 * k + 1] + lat[3 * k + 2] * lat[3 * k + 2]);
      if (!(len > 0)) return -1;
      int m = span == 0 ? (int)ceil(rc / len) : span;
      lo[k] = -m;
      hi[k] = m;
      for (int l = 0; l < k; ++l) {
        double dot = lat[3 * k] * lat[3 * l] + lat[3 * k + 1] * lat[3 * l + 1] + lat[3 * k + 2] * lat[3 * l + 2];
        int l_rot = 0;
        if (rot)
          for (int i = 0; i < 9; ++i)
            if (rot[9 * l + i] != ((i % 4 == 0) ? 1.0 : 0.0)) l_rot = 1;
        if (!l_rot && fabs(dot) > 1e-12 * len * len) return -1; /* orthogonal translations only */
      }
    }
  }
  /* the generators must commute */
  for (int k = 0; k < nper; ++k)
    for (int l = 0; l < k; ++l) {
      oc_xf a, b, ab, ba;
      oc_generator(lat, rot, k, 0, &a);
      oc_generator(lat, rot, l, 0, &b);
      oc_xf_compose(&a, &b, &ab);
      oc_xf_compose(&b, &a, &ba);
      for (int i = 0; i < 9; ++i)
        if (fabs(ab.R[i] - ba.R[i]) > 1e-12) return -1;
      for (int q = 0; q < 3; ++q)
        if (fabs(ab.y[q] - ba.y[q]) > 1e-9 * scale) return -1;
    }
  int cnt = 0;
  for (int a = lo[0]; a <= hi[0]; ++a)
    for (int b = lo[1]; b <= hi[1]; ++b)
      for (int c = lo[2]; c <= hi[2]; ++c) {
        int n[3] = {a, b, c};
        if (cnt >= maxn) return -1;
        oc_xf t;
        oc_xf_identity(&t);
        for (int k = 0; k < nper; ++k) {
          oc_xf g;
          oc_generator(lat, rot, k, n[k] < 0, &g);
          for (int r = 0; r < abs(n[k]); ++r) oc_xf_compose(&g, &t, &t);
        }
        for (int q = 0; q < 3; ++q) t.n[q] = n[q];
        out[cnt++] = t;
      }
  /* distinct images only (a generator power must not equal another image) */
  for (int i = 0; i < cnt; ++i)
    for (int j = 0; j < i; ++j) {
      int same = 1;
      for (int e = 0; e < 9 && same; ++e)
        if (fabs(out[i].R[e] - out[j].R[e]) > 1e-12) same = 0;
      for (int q = 0; q < 3 && same; ++q)
        if (fabs(out[i].y[q] - out[j].y[q]) > 1e-9 * scale) same = 0;
      if (same) return -1;
    }
  return cnt;
}

static int oc_is_zero(const int *n) { return n[0] == 0 && n[1] == 0 && n[2] == 0; }

#define OC_MAXIMG 4096
static oc_xf *oc_images_for(int nper, const double *lat, const double *rot, double rc, int span, int *count) {
  oc_xf *t = (oc_xf *)malloc(sizeof(oc_xf) * OC_MAXIMG);
  *count = oc_transforms(nper, lat, rot, rc, span, t, OC_MAXIMG);
  if (*count < 0) {
    free(t);
    return NULL;
  }
  return t;
}

/* ------------------------------------------------------------------ forces, energy, virial */

/* Row a collects sum over b, n with (b,n) != (a,0) and s < rc^2 of F_ab; U and W
 * collect half of each term per row (every pair is seen from both rows). */
static void oc_row(int64_t a, int64_t n, const double *x, const int32_t *sp, const double *eps, const double *sig,
                   double rc2, int nimg, const oc_xf *img, double *Fa, double *Ua, double *Wa, int64_t *npa) {
  double f0 = 0, f1 = 0, f2 = 0, u2 = 0, w2 = 0;
  int64_t cnt = 0;
  for (int64_t b = 0; b < n; ++b) {
    double e, sg;
    oc_mix(eps, sig, sp[a], sp[b], &e, &sg);
    for (int k = 0; k < nimg; ++k) {
      if (b == a && oc_is_zero(img[k].n)) continue;
      double xb[3];
      oc_xf_apply(&img[k], x + 3 * b, xb);
      double d0 = x[3 * a] - xb[0];
      double d1 = x[3 * a + 1] - xb[1];
      double d2 = x[3 * a + 2] - xb[2];
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
              double rc, int32_t nper, const double *lat, const double *rot, double *F, double *U, double *W,
              int64_t *npairs) {
  int nimg;
  oc_xf *img = oc_images_for(nper, lat, rot, rc, 0, &nimg);
  if (!img) return OC_E_INVAL;
  if (n < 0 || nsp < 1) {
    free(img);
    return OC_E_INVAL;
  }
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
  free(img);
  return OC_OK;
}

/* Forces on selected rows only (each against all n molecules): the sampled
 * check for workloads too large for all pairs.  Urow/Wrow/cnt are per-row half sums. */
int oc_forces_rows(int64_t n, const double *x, const int32_t *sp, int32_t nsp, const double *eps, const double *sig,
                   double rc, int32_t nper, const double *lat, const double *rot, int64_t nrows,
                   const int64_t *rows, double *F, double *Urow, double *Wrow, int64_t *cnt) {
  int nimg;
  oc_xf *img = oc_images_for(nper, lat, rot, rc, 0, &nimg);
  if (!img) return OC_E_INVAL;
  if (nsp < 1) {
    free(img);
    return OC_E_INVAL;
  }
  double rc2 = rc * rc;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < nrows; ++r) oc_row(rows[r], n, x, sp, eps, sig, rc2, nimg, img, F + 3 * r, Urow + r, Wrow + r, cnt + r);
  free(img);
  return OC_OK;
}

/* Pair set: every unordered pair {a, T_n b} with s < rc^2, reported as
 * (a, b, n) with a < b (or a == b and n lexicographically positive: a molecule
 * and its own image) and d = x_a - T_n x_b.  Returns the count; arrays may be
 * NULL to count only. */
int64_t oc_pairs(int64_t n, const double *x, double rc, int32_t nper, const double *lat, const double *rot,
                 int64_t cap, int32_t *pa, int32_t *pb, int8_t *pn) {
  int nimg;
  oc_xf *img = oc_images_for(nper, lat, rot, rc, 0, &nimg);
  if (!img) return -1;
  double rc2 = rc * rc;
  int64_t cnt = 0;
  for (int64_t a = 0; a < n; ++a)
    for (int64_t b = a; b < n; ++b)
      for (int k = 0; k < nimg; ++k) {
        const int *nk = img[k].n;
        if (b == a) { /* n lexicographically positive */
          int pos = 0;
          for (int q = 0; q < 3; ++q) {
            if (nk[q] > 0) {
              pos = 1;
              break;
            }
            if (nk[q] < 0) break;
          }
          if (!pos) continue;
        }
        double xb[3];
        oc_xf_apply(&img[k], x + 3 * b, xb);
        double d0 = x[3 * a] - xb[0];
        double d1 = x[3 * a + 1] - xb[1];
        double d2 = x[3 * a + 2] - xb[2];
        double s = d0 * d0 + d1 * d1 + d2 * d2;
        if (s < rc2) {
          if (pa && cnt < cap) {
            pa[cnt] = (int32_t)a;
            pb[cnt] = (int32_t)b;
            pn[3 * cnt] = (int8_t)nk[0];
            pn[3 * cnt + 1] = (int8_t)nk[1];
            pn[3 * cnt + 2] = (int8_t)nk[2];
          }
          ++cnt;
        }
      }
  free(img);
  return cnt;
}

/* ------------------------------------------------------------------ adjoint */

/* L = sum_i G_i . F_i + gamma U.  Per pair (a, b, image T) with d = x_a - T x_b, s = d.d, and the
 * image's G rotated with it, G_b' = R G_b (a force on the image acts on b rotated back by R^T):
 *   l = (G_a - G_b').d g(s) + gamma u(s)
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
 * Row a collects dL/dx_a = sum_b dl/dd(a,b) (each pair seen from both rows: from b's row the pair is
 * (b, a, T^-1) with d and G_a - G_b' both mapped by -R^T, and dl/dd maps the same way, so that row's
 * term is the gradient with respect to x_b); parameter sums take half per row. */
/* Row a of the adjoint: gxa = dL/dx_a; with pe, ps non-NULL, also the row's halves of the
 * species-pair sums of dl/deps_ab and dl/dsig_ab ([64], indexed 8 sp_a + sp_b) and of L. */
static void oc_adjoint_row(int64_t a, int64_t n, const double *x, const int32_t *sp, const double *eps,
                           const double *sig, double rc2, int nimg, const oc_xf *img, const double *G,
                           double gamma, double *gxa, double *pe, double *ps, double *pl) {
  double v0 = 0, v1 = 0, v2 = 0, la = 0;
  for (int64_t b = 0; b < n; ++b) {
    double e, sg;
    oc_mix(eps, sig, sp[a], sp[b], &e, &sg);
    for (int k = 0; k < nimg; ++k) {
      if (b == a && oc_is_zero(img[k].n)) continue;
      double xb[3], gb[3];
      oc_xf_apply(&img[k], x + 3 * b, xb);
      oc_xf_rotate(&img[k], G + 3 * b, gb);
      double dg0 = G[3 * a] - gb[0], dg1 = G[3 * a + 1] - gb[1], dg2 = G[3 * a + 2] - gb[2];
      double d0 = x[3 * a] - xb[0];
      double d1 = x[3 * a + 1] - xb[1];
      double d2 = x[3 * a + 2] - xb[2];
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
      if (!pe) continue;
      double l = gd * g + gamma * u;
      la += 0.5 * l;
      double dgds = (24.0 * e / sg) * (24.0 * sr12 - 6.0 * sr6) / s;
      double duds = (24.0 * e / sg) * (2.0 * sr12 - sr6);
      int t = sp[a] * 8 + sp[b];
      pe[t] += 0.5 * l / e;
      ps[t] += 0.5 * (gd * dgds + gamma * duds);
    }
  }
  gxa[0] = v0;
  gxa[1] = v1;
  gxa[2] = v2;
  if (pl) *pl = la;
}

int oc_adjoint(int64_t n, const double *x, const int32_t *sp, int32_t nsp, const double *eps, const double *sig,
               double rc, int32_t nper, const double *lat, const double *rot, const double *G, double gamma,
               double *gx, double *geps, double *gsig, double *L) {
  int nimg;
  oc_xf *img = oc_images_for(nper, lat, rot, rc, 0, &nimg);
  if (!img) return OC_E_INVAL;
  if (nsp < 1 || nsp > 8) {
    free(img);
    return OC_E_INVAL;
  }
  double rc2 = rc * rc;
  /* per-row partial sums for the species-pair parameter gradients and L */
  double *pe = (double *)calloc((size_t)(n > 0 ? n : 1) * 64, sizeof(double));
  double *ps = (double *)calloc((size_t)(n > 0 ? n : 1) * 64, sizeof(double));
  double *pl = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t a = 0; a < n; ++a)
    oc_adjoint_row(a, n, x, sp, eps, sig, rc2, nimg, img, G, gamma, gx + 3 * a, pe + 64 * a, ps + 64 * a, pl + a);
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
  free(img);
  return OC_OK;
}

/* dL/dx on selected rows only (each against all n molecules and images): the sampled check of the
 * adjoint for workloads too large for all pairs.  gx is [nrows][3]. */
int oc_adjoint_rows(int64_t n, const double *x, const int32_t *sp, int32_t nsp, const double *eps,
                    const double *sig, double rc, int32_t nper, const double *lat, const double *rot,
                    const double *G, double gamma, int64_t nrows, const int64_t *rows, double *gx) {
  int nimg;
  oc_xf *img = oc_images_for(nper, lat, rot, rc, 0, &nimg);
  if (!img) return OC_E_INVAL;
  if (nsp < 1 || nsp > 8) {
    free(img);
    return OC_E_INVAL;
  }
  double rc2 = rc * rc;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < nrows; ++r)
    oc_adjoint_row(rows[r], n, x, sp, eps, sig, rc2, nimg, img, G, gamma, gx + 3 * r, NULL, NULL, NULL);
  free(img);
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

/* Cell D mapped by the referring transform t: its vertices, triangles and bounding box (the caller
 * frees out->v and out->tri). */
static void oc_cell_mapped(const oc_cell *D, const oc_xf *t, oc_cell *out) {
  out->nv = D->nv;
  out->ntri = D->ntri;
  out->v = (double *)malloc(sizeof(double) * 3 * (D->nv > 0 ? D->nv : 1));
  out->tri = (double *)malloc(sizeof(double) * 9 * (D->ntri > 0 ? D->ntri : 1));
  for (int j = 0; j < D->nv; ++j) oc_xf_apply(t, D->v + 3 * j, out->v + 3 * j);
  for (int j = 0; j < 3 * D->ntri; ++j) oc_xf_apply(t, D->tri + 3 * j, out->tri + 3 * j);
  oc_xf_apply(t, D->cen, out->cen);
  for (int q = 0; q < 3; ++q) {
    out->lo[q] = 1e300;
    out->hi[q] = -1e300;
  }
  for (int j = 0; j < D->nv; ++j)
    for (int q = 0; q < 3; ++q) {
      if (out->v[3 * j + q] < out->lo[q]) out->lo[q] = out->v[3 * j + q];
      if (out->v[3 * j + q] > out->hi[q]) out->hi[q] = out->v[3 * j + q];
    }
}

static void oc_cell_unmap(oc_cell *c) {
  free(c->v);
  free(c->tri);
}

/* Is the closest distance between cell c and the (already mapped) cell d below R? */
static int oc_cells_in_range(const oc_cell *C, const oc_cell *D, double R) {
  double R2 = R * R;
  /* bounding boxes farther apart than R: not in range */
  double g2 = 0;
  for (int q = 0; q < 3; ++q) {
    double gap = 0;
    if (D->lo[q] > C->hi[q]) gap = D->lo[q] - C->hi[q];
    if (C->lo[q] > D->hi[q]) gap = C->lo[q] - D->hi[q];
    g2 += gap * gap;
  }
  if (g2 >= R2) return 0;
  /* a vertex pair closer than R: in range */
  for (int i = 0; i < C->nv; ++i)
    for (int j = 0; j < D->nv; ++j) {
      double d[3];
      sub3(C->v + 3 * i, D->v + 3 * j, d);
      if (dot3(d, d) < R2) return 1;
    }
  /* full minimum over boundary triangle pairs */
  for (int i = 0; i < C->ntri; ++i)
    for (int j = 0; j < D->ntri; ++j)
      if (tri_tri2(C->tri + 9 * i, D->tri + 9 * j) < R2) return 1;
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

/* Exact closest distance between cell c and cell d mapped by x -> Rm x + T (Rm NULL: the identity),
 * for pins. */
double oc_cell_distance(int64_t n_points, const double *points, int64_t n_faces, const int64_t *face_off,
                        const int32_t *face_pts, const int32_t *owner, const int32_t *neighbour, int64_t n_cells,
                        int32_t c, int32_t d, const double *T, const double *Rm) {
  oc_mesh m;
  oc_mesh_from(n_points, points, n_faces, face_off, face_pts, owner, neighbour, n_cells, &m);
  oc_cell *cells;
  if (oc_build_cells(&m, &cells) != OC_OK) return -1;
  oc_xf t;
  oc_xf_identity(&t);
  for (int q = 0; q < 3; ++q) t.y[q] = T[q];
  if (Rm)
    for (int i = 0; i < 9; ++i) t.R[i] = Rm[i];
  oc_xf_set_rot(&t);
  oc_cell Dm;
  oc_cell_mapped(&cells[d], &t, &Dm);
  double best = 1e300;
  oc_cell *C = &cells[c];
  for (int i = 0; i < C->ntri; ++i)
    for (int j = 0; j < Dm.ntri; ++j) {
      double v = tri_tri2(C->tri + 9 * i, Dm.tri + 9 * j);
      if (v < best) best = v;
    }
  oc_cell_unmap(&Dm);
  oc_free_cells(cells, n_cells);
  return sqrt(best);
}

/* The paper's own cell-pair predicate (Sec. 2.2, App. A.1): some vertex of c and some vertex of the
 * mapped cell d are closer than R.  Brute force over all vertex pairs. */
static int oc_vertices_in_range(const oc_cell *c, const oc_cell *d, double R) {
  for (int i = 0; i < c->nv; ++i)
    for (int j = 0; j < d->nv; ++j) {
      double s = 0;
      for (int q = 0; q < 3; ++q) {
        double e = c->v[3 * i + q] - d->v[3 * j + q];
        s += e * e;
      }
      if (s < R * R) return 1;
    }
  return 0;
}

/* Brute-force interacting cell pairs: every (c, d, n) with the closest distance
 * between cell c and cell d mapped by image n (powers in {-1,0,1}) below
 * rc + guard (predicate 0), or some vertex pair closer than that (predicate 1,
 * the paper's test), reported once: c < d, or c == d with n lexicographically
 * positive.  Returns the count (arrays may be NULL to count only), or <0 on
 * error. */
int64_t oc_dil(int64_t n_points, const double *points, int64_t n_faces, const int64_t *face_off,
               const int32_t *face_pts, const int32_t *owner, const int32_t *neighbour, int64_t n_cells,
               int32_t nper, const double *lat, const double *rot, double rc, double guard, int32_t predicate,
               int64_t cap, int32_t *oc, int32_t *od, int8_t *on) {
  oc_mesh m;
  oc_mesh_from(n_points, points, n_faces, face_off, face_pts, owner, neighbour, n_cells, &m);
  double R = rc + guard;
  int nimg;
  oc_xf *img = oc_images_for(nper, lat, rot, R, 1, &nimg);
  if (!img) return OC_E_INVAL;
  oc_cell *cells;
  if (oc_build_cells(&m, &cells) != OC_OK) {
    free(img);
    return OC_E_MESH;
  }
  int64_t cnt = 0;
  for (int64_t c = 0; c < n_cells; ++c)
    for (int64_t d = c; d < n_cells; ++d)
      for (int im = 0; im < nimg; ++im) {
        const int *n = img[im].n;
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
        oc_cell Dm;
        oc_cell_mapped(&cells[d], &img[im], &Dm);
        const int hit = predicate == 1 ? oc_vertices_in_range(&cells[c], &Dm, R) : oc_cells_in_range(&cells[c], &Dm, R);
        oc_cell_unmap(&Dm);
        if (hit) {
          if (oc && cnt < cap) {
            oc[cnt] = (int32_t)c;
            od[cnt] = (int32_t)d;
            for (int k = 0; k < 3; ++k) on[3 * cnt + k] = (int8_t)n[k];
          }
          ++cnt;
        }
      }
  oc_free_cells(cells, n_cells);
  free(img);
  return cnt;
}

/* Cell pairs (c, d, n), any order, in range (closest distance below rc + guard) through an image with
 * some power outside {-1,0,1}: translations to +-2, rotations over their whole group.  Zero means the
 * first images suffice (the referred-cell lists with powers in {-1,0,1} are complete). */
int64_t oc_far_images(int64_t n_points, const double *points, int64_t n_faces, const int64_t *face_off,
                      const int32_t *face_pts, const int32_t *owner, const int32_t *neighbour, int64_t n_cells,
                      int32_t nper, const double *lat, const double *rot, double rc, double guard) {
  oc_mesh m;
  oc_mesh_from(n_points, points, n_faces, face_off, face_pts, owner, neighbour, n_cells, &m);
  double R = rc + guard;
  int nimg;
  oc_xf *img = oc_images_for(nper, lat, rot, R, 2, &nimg);
  if (!img) return OC_E_INVAL;
  oc_cell *cells;
  if (oc_build_cells(&m, &cells) != OC_OK) {
    free(img);
    return OC_E_MESH;
  }
  int64_t cnt = 0;
  for (int im = 0; im < nimg; ++im) {
    const int *n = img[im].n;
    if (abs(n[0]) <= 1 && abs(n[1]) <= 1 && abs(n[2]) <= 1) continue;
    for (int64_t d = 0; d < n_cells; ++d) {
      oc_cell Dm;
      oc_cell_mapped(&cells[d], &img[im], &Dm);
      for (int64_t c = 0; c < n_cells; ++c) cnt += oc_cells_in_range(&cells[c], &Dm, R);
      oc_cell_unmap(&Dm);
    }
  }
  oc_free_cells(cells, n_cells);
  free(img);
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
