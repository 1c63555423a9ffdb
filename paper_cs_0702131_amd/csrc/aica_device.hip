// HIP (gfx950) kernels and the C ABI of the AICA Lennard-Jones library.
//
// Per step (aica_bin, then aica_forces / aica_forces_adjoint):
//   locate -> histogram -> scan -> scatter -> in-cell sort     : CSR cell occupancy (Sec. 2.2)
//   group ranges, j-slot offsets                               : the per-step work list
//   gather                                                     : cell-sorted SoA, group-local coordinates
//   pair kernel                                                : real-real and periodic referred pairs,
//                                                                Newton reactions (Sec. 2.3.1, 2.3.2, 2.2)
//   finalize, reduce                                           : per-molecule sums in caller order, U, W
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>
#include <string>
#include <vector>

#include "aica_internal.h"
#include "aica_kernels.h"

namespace aica {
const char *last_error_cstr();
}

using namespace aica;

#define HIPCHK(x)                                                                                       \
  do {                                                                                                  \
    hipError_t _e = (x);                                                                                \
    if (_e != hipSuccess) return fail(AICA_E_HIP, std::string("HIP error: ") + hipGetErrorString(_e) + \
                                                      " at " + __FILE__ + ":" + std::to_string(__LINE__)); \
  } while (0)

namespace {

struct DBuf {
  void *p = nullptr;
  size_t bytes = 0;
  ~DBuf() {
    if (p) (void)hipFree(p);
  }
  int ensure(size_t nbytes) {
    if (nbytes <= bytes && p) return AICA_OK;
    if (p) {
      (void)hipFree(p);
      p = nullptr;
      bytes = 0;
    }
    size_t nb = std::max<size_t>(nbytes, 256);
    if (hipMalloc(&p, nb) != hipSuccess) {
      p = nullptr;
      return fail(AICA_E_NOMEM, "device allocation of " + std::to_string(nb) + " bytes failed");
    }
    bytes = nb;
    return AICA_OK;
  }
  template <class T>
  T *as() const {
    return (T *)p;
  }
  void swap(DBuf &o) {
    std::swap(p, o.p);
    std::swap(bytes, o.bytes);
  }
};

template <class T>
int upload(DBuf &b, const std::vector<T> &v) {
  int rc = b.ensure(sizeof(T) * std::max<size_t>(v.size(), 1));
  if (rc) return rc;
  if (!v.empty()) HIPCHK(hipMemcpy(b.p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  return AICA_OK;
}

struct Timer {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  double ms = 0;
  int64_t launches = 0;
};

}  // namespace

struct aica_dil {
  Geometry geo;
  std::vector<int32_t> order, rank;
  std::vector<uint8_t> split_depth;  // k-d tree of the sorted order (groups are its subtrees)
  std::vector<CellPair> pairs;
  double rcut = 0, guard = 0, build_seconds = 0, group_seconds = 0;
  int device = 0;
  bool geometry_on_device = false;
  // device geometry for point location (mesh cell ids)
  DBuf d_rec_off, d_rec, d_bb;  // point-location cell records and padded boxes, sorted cell order
  DBuf d_rec32;                 // FP32 records for the previous-cell test (cells of at most kR32 float4)
  DBuf d_pl32;                  // plane records of the boundary triangles (kPl float4 per cell, with d_rec32)
  DBuf d_nbr_off, d_nbr;        // cells across each cell's interior faces (sorted ids)
  bool has_rec32 = false;
  DBuf d_gb_off, d_gb_cell;
  double glo[3] = {0, 0, 0}, gh = 1;
  int64_t gnb[3] = {1, 1, 1};
  // interaction groups (depend on the number density; built on the first aica_bin)
  bool groups_ready = false;
  int64_t groups_for_n = -1;
  Groups grp;
  DBuf d_orig, d_g_cell0, d_e_off, d_e_B, d_e_vec32, d_e_vec64, d_nl_off, d_nl_e, d_nl_d, d_nl_r, d_rcnt;
  DBuf d_rot64;                 // [27][9] rotation of every image code (only with rotational referral)
  // per step
  bool bin_valid = false;
  bool wsteps_valid = false;  // d_gnp holds the wave-step counts of a forward call on the current binning
  int64_t n = 0;
  const void *bin_pos = nullptr;
  int32_t bin_dtype = 0;
  int64_t jtotal = 0;
  DBuf d_cell_of, d_count, d_cell_start, d_rank, d_perm, d_g_start, d_mol_group, d_jcnt, d_slot_base, d_cell_sorted;
  DBuf d_scan_tmp, d_status, d_slow;
  DBuf d_ref;                   // [n] float4 per caller molecule id: centre and radius of a ball that lies
                                // inside the molecule's cell of the last binning (radius 0: none)
  DBuf d_perm_prev;     // the previous binning's permutation during aica_bin
  int64_t perm_n = -1;  // molecule count of the binning held in d_perm and d_cell_sorted (-1: none)
  int64_t located[3] = {0, 0, 0};  // last binning: molecules located by their ball, by the FP32 record, slowly
  // force / adjoint workspace
  DBuf d_pos, d_own, d_jpart, d_gpart, d_gnp, d_gG, d_gpar;
  DBuf d_pairs, d_pcount;
  DBuf d_red;  // stage-1 rows of the group reductions
  bool profiling = false;
  uint32_t epoch = 0;          // tag of the reaction records written by the current call
  size_t jpart_tagged = 0;     // bytes of d_jpart known to hold no valid tag
  std::map<std::string, Timer> timers;
};

// =====================================================================================================
// kernels: binning

namespace {

__device__ __forceinline__ double orient3(const double *a, const double *b, const double *c, const double *d) {
  const double u0 = b[0] - a[0], u1 = b[1] - a[1], u2 = b[2] - a[2];
  const double v0 = c[0] - a[0], v1 = c[1] - a[1], v2 = c[2] - a[2];
  const double w0 = d[0] - a[0], w1 = d[1] - a[1], w2 = d[2] - a[2];
  return u0 * (v1 * w2 - v2 * w1) + u1 * (v2 * w0 - v0 * w2) + u2 * (v0 * w1 - v1 * w0);
}

// Cell records for point location, one per sorted cell, contiguous:
//   [nf, cc(3), fc_0(3) .. fc_{nf-1}(3), len_0 .. len_{nf-1}, loop_0(3 len_0) .. loop_{nf-1}(3 len_{nf-1})]
// with cc the cell's vertex mean, fc the face centroids and each face's vertex loop oriented outward
// from the cell (counts stored as doubles, exact).
//
// Is p inside the cell: some tetrahedron (cc, fc, v_k, v_k+1) contains p, with a relative tolerance tau
// of that tetrahedron's volume (tau = 1e-12 for membership; the previous-cell fast path asks for
// tau = -1e-9, i.e. strictly inside).  The four barycentric tests of tetrahedron k are: the outer face,
// orient(p, fc, v_k, v_k+1) >= -tol; the edge plane through cc, orient(cc, p, v_k, v_k+1) >= -tol; and
// the two spoke planes (cc, fc, v_k), (cc, fc, v_k+1), whose orientations s_k = orient(cc, fc, v_k, p)
// are shared by neighbouring tetrahedra of the fan.  The face whose centroid direction from cc best
// matches p - cc is tried first (the answer does not depend on the order).
__device__ bool point_in_face_fan(const double *p, const double *cc, const double *fc, const double *V, int len,
                                  double tau) {
  double s_first = orient3(cc, fc, V, p), s_prev = s_first;
  const double *vp = V;
  for (int j = 0; j < len; ++j) {
    const double *vn = V + 3 * (j + 1 == len ? 0 : j + 1);
    const double s_next = (j + 1 == len) ? s_first : orient3(cc, fc, vn, p);
    const double v = orient3(cc, fc, vp, vn);
    const double tol = -tau * fabs(v);
    if (s_prev >= tol && -s_next >= tol && orient3(p, fc, vp, vn) >= tol && orient3(cc, p, vp, vn) >= tol)
      return true;
    s_prev = s_next;
    vp = vn;
  }
  return false;
}

__device__ bool point_in_rec(const double *p, const double *R, double tau) {
  const int nf = (int)R[0];
  const double *cc = R + 1, *FC = R + 4, *LEN = FC + 3 * nf, *V = LEN + nf;
  const double d0 = p[0] - cc[0], d1 = p[1] - cc[1], d2 = p[2] - cc[2];
  int best = 0;
  double bs = -1e300;
  int64_t boff = 0, off = 0;
  for (int k = 0; k < nf; ++k) {
    const double e0 = FC[3 * k] - cc[0], e1 = FC[3 * k + 1] - cc[1], e2 = FC[3 * k + 2] - cc[2];
    const double sc = (d0 * e0 + d1 * e1 + d2 * e2) / (e0 * e0 + e1 * e1 + e2 * e2);
    if (sc > bs) {
      bs = sc;
      best = k;
      boff = off;
    }
    off += 3 * (int64_t)LEN[k];
  }
  if (point_in_face_fan(p, cc, FC + 3 * best, V + boff, (int)LEN[best], tau)) return true;
  off = 0;
  for (int k = 0; k < nf; ++k) {
    const int len = (int)LEN[k];
    if (k != best && point_in_face_fan(p, cc, FC + 3 * k, V + off, len, tau)) return true;
    off += 3 * (int64_t)len;
  }
  return false;
}

// FP32 copies of the cell records for the previous-cell test, fixed stride kR32 float4 per sorted cell:
//   [0] (nf, a.x, a.y, a.z) with a the FP32-rounded vertex mean; [1] (cc - a, 0);
//   [2 .. 2 + nf) (fc_k - a, len_k); then the face loops, one vertex (v - a, 0) per float4, except that the
//   first vertex of face k's loop carries in .w the sorted id of the cell across face k (int bits; -1 on
//   a boundary face).
// A point is accepted when some tetrahedron contains it with every orientation above 1e-4 of that
// tetrahedron's own (FP32) orientation.  The FP32 rounding of the records and of the orientations is
// below 1e-5 of that scale, so an accepted point is strictly inside in exact arithmetic too (the FP64
// test with tau = -1e-9 accepts it); anything else goes to the FP64 test.
constexpr int kR32 = 32;

__device__ __forceinline__ float orient3f(const float *a, const float *b, const float *c, const float *d) {
  const float u0 = b[0] - a[0], u1 = b[1] - a[1], u2 = b[2] - a[2];
  const float v0 = c[0] - a[0], v1 = c[1] - a[1], v2 = c[2] - a[2];
  const float w0 = d[0] - a[0], w1 = d[1] - a[1], w2 = d[2] - a[2];
  return u0 * (v1 * w2 - v2 * w1) + u1 * (v2 * w0 - v0 * w2) + u2 * (v0 * w1 - v1 * w0);
}

// across (optional): the sorted id of the cell across the face whose centroid direction best matches
// p - cc (the face a molecule that left the cell has most likely crossed), -1 on a boundary face.
__device__ bool surely_in_rec32(const double *p, const float4 *R, int *across = nullptr) {
  const float4 h = R[0], h2 = R[1];
  const int nf = (int)h.x;
  const float pr[3] = {(float)(p[0] - (double)h.y), (float)(p[1] - (double)h.z), (float)(p[2] - (double)h.w)};
  const float cc[3] = {h2.x, h2.y, h2.z};
  // best face first (the answer does not depend on the order)
  int best = 0, boff = 0, off = 0;
  float bs = -3.0e38f;
  for (int k = 0; k < nf; ++k) {
    const float4 f = R[2 + k];
    const float e0 = f.x - cc[0], e1 = f.y - cc[1], e2 = f.z - cc[2];
    const float sc = ((pr[0] - cc[0]) * e0 + (pr[1] - cc[1]) * e1 + (pr[2] - cc[2]) * e2) / (e0 * e0 + e1 * e1 + e2 * e2);
    if (sc > bs) {
      bs = sc;
      best = k;
      boff = off;
    }
    off += (int)f.w;
  }
  if (across) *across = __float_as_int(R[2 + nf + boff].w);
  auto fan = [&](int k, int voff) -> bool {
    const float4 f = R[2 + k];
    const float fc[3] = {f.x, f.y, f.z};
    const int len = (int)f.w;
    const float4 *V = R + 2 + nf + voff;
    float vp[3] = {V[0].x, V[0].y, V[0].z};
    const float s_first = orient3f(cc, fc, vp, pr);
    float s_prev = s_first;
    for (int j = 0; j < len; ++j) {
      const float4 n4 = V[j + 1 == len ? 0 : j + 1];
      const float vn[3] = {n4.x, n4.y, n4.z};
      const float s_next = (j + 1 == len) ? s_first : orient3f(cc, fc, vn, pr);
      const float tol = 1e-4f * fabsf(orient3f(cc, fc, vp, vn));
      if (s_prev > tol && -s_next > tol && orient3f(pr, fc, vp, vn) > tol && orient3f(cc, pr, vp, vn) > tol)
        return true;
      s_prev = s_next;
      vp[0] = vn[0];
      vp[1] = vn[1];
      vp[2] = vn[2];
    }
    return false;
  };
  if (fan(best, boff)) return true;
  off = 0;
  for (int k = 0; k < nf; ++k) {
    const int len = (int)R[2 + k].w;
    if (k != best && fan(k, off)) return true;
    off += len;
  }
  return false;
}

// Radius of a ball about p that lies inside the cell of FP32 record R, for a p that the record shows
// strictly inside: the cell's boundary is made of the face-fan triangles, and the distance from p to a
// triangle is at least the distance to its plane, so the smallest plane distance bounds the distance to
// the boundary from below.  FP32 rounding is covered by a margin of 1e-4 of the cell's size.  Returns the
// ball as (centre rounded to FP32, radius reduced by that rounding); radius 0 when nothing is left.
__device__ float4 inner_ball(const double *p, const float4 *R) {
  const float4 h = R[0], h2 = R[1];
  const int nf = (int)h.x;
  const float pr[3] = {(float)(p[0] - (double)h.y), (float)(p[1] - (double)h.z), (float)(p[2] - (double)h.w)};
  float dmin = 3.0e38f, size = 0.f;
  int off = 0;
  for (int k = 0; k < nf; ++k) {
    const float4 f = R[2 + k];
    const int len = (int)f.w;
    const float e0 = f.x - h2.x, e1 = f.y - h2.y, e2 = f.z - h2.z;
    size = fmaxf(size, sqrtf(e0 * e0 + e1 * e1 + e2 * e2));
    const float4 *V = R + 2 + nf + off;
    for (int j = 0; j < len; ++j) {
      const float4 va = V[j], vb = V[j + 1 == len ? 0 : j + 1];
      const float a0 = va.x - f.x, a1 = va.y - f.y, a2 = va.z - f.z;
      const float b0 = vb.x - f.x, b1 = vb.y - f.y, b2 = vb.z - f.z;
      const float n0 = a1 * b2 - a2 * b1, n1 = a2 * b0 - a0 * b2, n2 = a0 * b1 - a1 * b0;
      const float nn = sqrtf(n0 * n0 + n1 * n1 + n2 * n2);
      const float dd = fabsf(n0 * (pr[0] - f.x) + n1 * (pr[1] - f.y) + n2 * (pr[2] - f.z));
      if (nn > 0.f) dmin = fminf(dmin, dd / nn);
      else dmin = 0.f;
    }
    off += len;
  }
  const float pc[3] = {(float)p[0], (float)p[1], (float)p[2]};
  const double s0 = p[0] - (double)pc[0], s1 = p[1] - (double)pc[1], s2 = p[2] - (double)pc[2];
  const double r = (double)dmin * (1.0 - 1e-6) - 1e-4 * (double)size - sqrt(s0 * s0 + s1 * s1 + s2 * s2);
  return make_float4(pc[0], pc[1], pc[2], r > 0 ? (float)r : 0.f);
}

// Plane records: per sorted cell kPl float4 (n, d), one per boundary triangle of the cell's face fans: the
// inward unit normal n and d = n.(f - a) for a point f of the triangle, in the frame a of the cell's FP32
// record, so that n.(p - a) - d is the signed distance of p from the triangle's plane (positive inside).
// Unused entries are (0, 0, 0, -3e38); a cell with more triangles than kPl has (0, 0, 0, 3e38) in entry 0,
// so that its test never accepts.
constexpr int kPl = 24;

// A point on the inner side of every boundary triangle's plane is strictly inside the cell: from a point
// outside the cell (or on its boundary), a segment to an interior point enters the cell through some
// boundary triangle, so that point lies on the outer side of (or on) the triangle's plane.  Accepts p when
// the smallest signed distance exceeds 1e-4 of the cell's size (the FP32 rounding of the planes, of p - a
// and of the sums is below 1e-6 of it), and gives the ball about p (centre rounded to FP32) that stays
// inside: radius = that distance less the margin and the centre's rounding.  A point inside but not this
// far from every plane (near the boundary, or beside a reflex crease of a non-convex cell) is left to the
// fan test.
__device__ bool plane_ball(const double *p, const float4 *R, const float4 *PL, float4 &ball) {
  const float4 h = R[0];
  const float size = R[1].w;
  const float pr0 = (float)(p[0] - (double)h.y), pr1 = (float)(p[1] - (double)h.z), pr2 = (float)(p[2] - (double)h.w);
  float smin = 3.0e38f;
#pragma unroll 8
  for (int k = 0; k < kPl; ++k) {
    const float4 q = PL[k];
    smin = fminf(smin, fmaf(q.x, pr0, fmaf(q.y, pr1, fmaf(q.z, pr2, -q.w))));
  }
  if (!(smin > 1e-4f * size)) return false;
  const float pc[3] = {(float)p[0], (float)p[1], (float)p[2]};
  const double s0 = p[0] - (double)pc[0], s1 = p[1] - (double)pc[1], s2 = p[2] - (double)pc[2];
  const double r = (double)smin * (1.0 - 1e-6) - 1e-4 * (double)size - sqrt(s0 * s0 + s1 * s1 + s2 * s2);
  ball = make_float4(pc[0], pc[1], pc[2], r > 0 ? (float)r : 0.f);
  return true;
}

// Locate each molecule: cell_of[i] = sorted index of the cell that contains x_i, in two kernels so that
// the rare slow cases do not hold up whole waves.
// k_locate_fast visits molecules in the order trav (the previous binning's sorted order, so that
// neighbouring threads read neighbouring cell records), kLocPerLane per lane: a molecule still inside the
// ball kept from its last record test is in its previous cell (hint); the others are compacted in LDS and
// tested 64 at a time against the FP32 records (the previous cell, then the cell across the face most
// likely crossed: a molecule that a record shows strictly inside a cell is in no other); every other
// molecule goes to a list.  k_locate_slow takes that list, a group of lanes per molecule: the FP64 previous-cell
// test and the cells across the previous cell's faces (a molecule that left its cell has crossed one of
// them: the paper's membership tracking), each accepted only when the point is strictly inside; then
// every cell whose padded box holds the point, in ascending mesh cell id (the lowest containing cell wins
// a tie on a shared face, edge or vertex).  Without FP32 records (a cell too large for the fixed stride)
// or without a previous binning every molecule takes the slow path.
// Both kernels index their state by t, the molecule's slot in the previous binning's sorted order
// (trav[t] = its caller index, hint[t] = its previous cell; without a previous binning t is the
// caller index and there is no hint), so that only the positions are read out of order.
constexpr int kRouteSlots = 64;

constexpr int kLocPerLane = 4;  // molecules per lane in the fast kernel

template <typename PT>
__global__ __launch_bounds__(256) void k_locate_fast(
    const PT *__restrict__ pos, int64_t n, const int32_t *__restrict__ trav, const int32_t *__restrict__ hint,
    const float4 *__restrict__ rec32, const float4 *__restrict__ pl32, float4 *__restrict__ ref,
    int32_t *__restrict__ cell_t, int32_t *__restrict__ rank_t, int32_t *__restrict__ count,
    unsigned long long *__restrict__ nslow, int32_t *__restrict__ slow, unsigned long long *__restrict__ routes) {
  constexpr int kSpan = 64 * kLocPerLane;  // molecules per wave
  __shared__ int32_t rec_l[4][kSpan];      // per wave: slots (relative to the wave's first) for the records
  __shared__ int32_t slow_l[4][kSpan];     // per wave: slots for the slow kernel
  const int lane = (int)(threadIdx.x & 63), w = (int)(threadIdx.x >> 6);
  const int64_t base = ((int64_t)blockIdx.x * 4 + w) * kSpan;
  int nr = 0, ns = 0;  // wave-uniform list lengths
  auto push = [&](int32_t *L, int &len, bool take, int val) {
    const unsigned long long m = __builtin_amdgcn_ballot_w64(take);
    if (take) L[len + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u))] = val;
    len += (int)__builtin_popcountll(m);
  };
  // ---- the ball test, kLocPerLane molecules per lane
  for (int k = 0; k < kLocPerLane; ++k) {
    const int off = k * 64 + lane;
    const int64_t t = base + off;
    int how = -1;  // 0: inside its ball, 1: to the record test, 2: to the slow kernel
    if (t < n) {
      const int64_t i = trav ? trav[t] : t;
      const double p[3] = {(double)pos[3 * i], (double)pos[3 * i + 1], (double)pos[3 * i + 2]};
      const int32_t h0 = hint ? hint[t] : -1;
      how = 2;
      if (h0 >= 0 && isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2])) {
        // still inside the ball found inside this cell when it was last tested: no record needed
        const float4 b = ref[i];
        const double e0 = p[0] - (double)b.x, e1 = p[1] - (double)b.y, e2 = p[2] - (double)b.z;
        if (b.w > 0.f && e0 * e0 + e1 * e1 + e2 * e2 < (double)b.w * (double)b.w) {
          how = 0;
          cell_t[t] = h0;
          rank_t[t] = atomicAdd(&count[h0], 1);
        } else if (rec32) {
          how = 1;
        }
      }
    }
    push(rec_l[w], nr, how == 1, off);
    push(slow_l[w], ns, how == 2, off);
  }
  wave_lds_sync();
  // ---- the FP32 records of the molecules that left their ball, 64 at a time on a compacted list: the
  // previous cell, then the cell across the face most likely crossed
  int nrec = 0;
  for (int b = 0; b < nr; b += 64) {
    int how = -1;
    int off = 0;
    if (b + lane < nr) {
      off = rec_l[w][b + lane];
      const int64_t t = base + off;
      const int64_t i = trav[t];
      const double p[3] = {(double)pos[3 * i], (double)pos[3 * i + 1], (double)pos[3 * i + 2]};
      const int32_t h0 = hint[t];
      int32_t found = -1, across = -1;
      float4 ball;
      bool have_ball = false;  // the plane test accepted and gave the ball
      if (pl32 && plane_ball(p, rec32 + (int64_t)kR32 * h0, pl32 + (int64_t)kPl * h0, ball)) {
        found = h0;
        have_ball = true;
      } else if (surely_in_rec32(p, rec32 + (int64_t)kR32 * h0, &across)) {
        found = h0;
      } else if (across >= 0) {
        if (pl32 && plane_ball(p, rec32 + (int64_t)kR32 * across, pl32 + (int64_t)kPl * across, ball)) {
          found = across;
          have_ball = true;
        } else if (surely_in_rec32(p, rec32 + (int64_t)kR32 * across)) {
          found = across;
        }
      }
      if (found >= 0) {
        how = 1;
        ref[i] = have_ball ? ball : inner_ball(p, rec32 + (int64_t)kR32 * found);
        cell_t[t] = found;
        rank_t[t] = atomicAdd(&count[found], 1);
      } else {
        how = 2;
      }
    }
    nrec += (int)__builtin_popcountll(__builtin_amdgcn_ballot_w64(how == 1));
    push(slow_l[w], ns, how == 2, off);
  }
  wave_lds_sync();
  // ---- the wave's share of the slow list (one atomic), and of the route counters (spread over
  // kRouteSlots addresses so that the waves do not queue on one)
  if (ns > 0) {
    unsigned long long start = 0;
    if (lane == 0) start = atomicAdd(nslow, (unsigned long long)ns);
    start = __shfl(start, 0, 64);
    for (int b = lane; b < ns; b += 64) slow[start + b] = (int32_t)(base + slow_l[w][b]);
  }
  if (lane == 0 && nrec > 0)
    atomicAdd(routes + (blockIdx.x * 4 + w) % kRouteSlots, (unsigned long long)nrec);
}

// The slow path for one molecule at p with previous cell h0 (-1: none): the previous cell and the cells
// across its faces, each accepted only when p is strictly inside (so at most one accepts), then the cells of
// the background bin whose padded box holds p, in ascending mesh cell id, the first containing one.  LANES
// (16 or 64) > 1: a group of that many lanes (a whole wave, or four molecules per wave) tests that many
// candidates side by side (the lowest accepting lane is the first accepting candidate, so the answer is that
// of testing them one after another); every branch below depends only on values shared by the group, so its
// lanes stay together.  With FP32 records the cells across the faces are first tried with the FP32 test,
// which only accepts points strictly inside.  LANES = 1: one lane tests the candidates in turn.
template <int LANES>
__device__ int32_t slow_find(const double *p, int32_t h0, const float4 *__restrict__ rec32, const float4 *__restrict__ pl32,
                             const int64_t *__restrict__ rec_off, const double *__restrict__ rec,
                             const int64_t *__restrict__ nbr_off, const int32_t *__restrict__ nbr,
                             const double *__restrict__ bb, const int64_t *__restrict__ gb_off,
                             const int32_t *__restrict__ gb_cell, double glo0, double glo1, double glo2, double gh,
                             int64_t nb0, int64_t nb1, int64_t nb2) {
  constexpr bool WAVE = LANES > 1;
  constexpr int kStep = LANES;
  const int lane = WAVE ? (int)(threadIdx.x & (LANES - 1)) : 0;
  const int g0lane = WAVE ? (int)(threadIdx.x & 63) - lane : 0;  // first lane of this molecule's group
  int32_t found = -1;
  // one round of candidate tests: k-th candidate c(k) for k < kc, test(c) -> accepted
  auto round = [&](int64_t b, int64_t kc, auto cand, auto test) {
    const int64_t k = b + lane;
    int32_t c = -1;
    bool in = false;
    if (k < kc) {
      c = cand(k);
      in = test(c);
    }
    if constexpr (WAVE) {
      const unsigned long long m =
          LANES == 64 ? __builtin_amdgcn_ballot_w64(in) : (__builtin_amdgcn_ballot_w64(in) >> g0lane) & ((1ull << LANES) - 1);
      if (m) found = __shfl(c, g0lane + (int)__builtin_ctzll(m), 64);
    } else if (in) {
      found = c;
    }
  };
  if (h0 >= 0) {
    const int64_t k0 = nbr_off[h0], kc = nbr_off[h0 + 1] - k0 + 1;  // the previous cell and its neighbours
    auto cand = [&](int64_t k) { return k == 0 ? h0 : nbr[k0 + k - 1]; };
    float4 ball;
    if (WAVE && pl32)
      for (int64_t b = 0; b < kc && found < 0; b += kStep)
        round(b, kc, cand, [&](int32_t c) { return plane_ball(p, rec32 + (int64_t)kR32 * c, pl32 + (int64_t)kPl * c, ball); });
    if (WAVE && rec32)
      for (int64_t b = 0; b < kc && found < 0; b += kStep)
        round(b, kc, cand, [&](int32_t c) { return surely_in_rec32(p, rec32 + (int64_t)kR32 * c); });
    for (int64_t b = 0; b < kc && found < 0; b += kStep)
      round(b, kc, cand, [&](int32_t c) { return point_in_rec(p, rec + rec_off[c], -1e-9); });
  }
  if (found < 0) {
    const double f0 = floor((p[0] - glo0) / gh), f1 = floor((p[1] - glo1) / gh), f2 = floor((p[2] - glo2) / gh);
    if (f0 >= 0 && f1 >= 0 && f2 >= 0 && f0 < (double)nb0 && f1 < (double)nb1 && f2 < (double)nb2) {
      const int64_t bin = (int64_t)f0 + nb0 * ((int64_t)f1 + nb1 * (int64_t)f2);
      const int64_t g0 = gb_off[bin], g1 = gb_off[bin + 1];
      // a cell whose planes show the point strictly inside is the only cell that holds it
      if (pl32) {
        float4 ball;
        for (int64_t b = 0; b < g1 - g0 && found < 0; b += kStep)
          round(b, g1 - g0, [&](int64_t k) { return gb_cell[g0 + k]; }, [&](int32_t c) {
            const double *B = bb + 6 * (int64_t)c;
            if (p[0] < B[0] || p[1] < B[1] || p[2] < B[2] || p[0] > B[3] || p[1] > B[4] || p[2] > B[5]) return false;
            return plane_ball(p, rec32 + (int64_t)kR32 * c, pl32 + (int64_t)kPl * c, ball);
          });
      }
      for (int64_t b = 0; b < g1 - g0 && found < 0; b += kStep)
        round(b, g1 - g0, [&](int64_t k) { return gb_cell[g0 + k]; }, [&](int32_t c) {
          const double *B = bb + 6 * (int64_t)c;
          if (p[0] < B[0] || p[1] < B[1] || p[2] < B[2] || p[0] > B[3] || p[1] > B[4] || p[2] > B[5]) return false;
          return point_in_rec(p, rec + rec_off[c], 1e-12);
        });
    }
  }
  return found;
}

// The slow kernel.  Molecules that have a previous cell: LANES (16 or 64) lanes per molecule; otherwise (the
// first binning, where every molecule comes here) LANES = 1, one thread per molecule.  A fixed grid strides
// over the list, whose length is only known on the device.  A group of 16 lanes keeps four molecules in
// flight per wave, which pays when the list is longer than the grid's waves; with fewer molecules a whole
// wave per molecule ends sooner (a wave of four molecules runs their different paths one after another).
template <typename PT, int LANES>
__global__ __launch_bounds__(256) void k_locate_slow(
    const PT *__restrict__ pos, const unsigned long long *__restrict__ nslow, const int32_t *__restrict__ slow,
    const int32_t *__restrict__ trav, const int32_t *__restrict__ hint, const float4 *__restrict__ rec32,
    const float4 *__restrict__ pl32, const int64_t *__restrict__ rec_off, const double *__restrict__ rec,
    const int64_t *__restrict__ nbr_off,
    const int32_t *__restrict__ nbr, const double *__restrict__ bb, const int64_t *__restrict__ gb_off,
    const int32_t *__restrict__ gb_cell, double glo0, double glo1, double glo2, double gh, int64_t nb0, int64_t nb1,
    int64_t nb2, float4 *__restrict__ ref, int32_t *__restrict__ cell_t, int32_t *__restrict__ rank_t,
    int32_t *__restrict__ count, unsigned long long *__restrict__ status) {
  const int64_t ns = (int64_t)*nslow;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, gsize = (int64_t)gridDim.x * blockDim.x;
  constexpr int kSh = __builtin_ctz(LANES);
  const int64_t u0 = gid >> kSh, ustep = gsize >> kSh;
  for (int64_t u = u0; u < ns; u += ustep) {  // uniform in each lane group
    const int64_t t = slow[u];
    const int64_t i = trav ? trav[t] : t;
    const double p[3] = {(double)pos[3 * i], (double)pos[3 * i + 1], (double)pos[3 * i + 2]};
    int32_t found = -1;
    if (isfinite(p[0]) && isfinite(p[1]) && isfinite(p[2]))
      found = slow_find<LANES>(p, hint ? hint[t] : -1, rec32, pl32, rec_off, rec, nbr_off, nbr, bb, gb_off, gb_cell, glo0,
                              glo1, glo2, gh, nb0, nb1, nb2);
    if ((threadIdx.x & (LANES - 1)) == 0) {
      cell_t[t] = found;
      // the ball about p inside the cell found, when the plane test shows p that far inside; else no ball
      // until the next record test in this cell
      float4 ball = make_float4(0.f, 0.f, 0.f, 0.f);
      if (found >= 0 && pl32) {
        float4 b;
        if (plane_ball(p, rec32 + (int64_t)kR32 * found, pl32 + (int64_t)kPl * found, b)) ball = b;
      }
      ref[i] = ball;
      if (found < 0)
        atomicAdd(status, 1ull);
      else
        rank_t[t] = atomicAdd(&count[found], 1);
    }
  }
}


// ---- exclusive scan of int32 counts into OutT offsets (out[n] = total)

constexpr int kScanThreads = 1024, kScanItems = 4, kScanTile = kScanThreads * kScanItems;

template <typename OutT>
__device__ OutT block_exclusive_scan(OutT v, OutT *sh, OutT &total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  OutT x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    OutT y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  if (w == 0) {
    OutT s = lane < (kScanThreads / 64) ? sh[lane] : 0;
    OutT t = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      OutT y = __shfl_up(t, o, 64);
      if (lane >= o) t += y;
    }
    if (lane < kScanThreads / 64) sh[lane] = t - s;
    if (lane == kScanThreads / 64 - 1) sh[kScanThreads / 64] = t;
  }
  __syncthreads();
  total = sh[kScanThreads / 64];
  OutT r = x - v + sh[w];
  __syncthreads();
  return r;
}

template <typename InT, typename OutT>
__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(const InT *in, int64_t n, OutT *out, OutT *tile_sum) {
  __shared__ OutT sh[kScanThreads / 64 + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  OutT v[kScanItems], s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? (OutT)in[base + k] : 0;
    s += v[k];
  }
  OutT total;
  OutT ex = block_exclusive_scan<OutT>(s, sh, total);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = ex;
    ex += v[k];
  }
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

template <typename OutT>
__global__ __launch_bounds__(kScanThreads) void k_scan_sums(OutT *tile_sum, int64_t ntiles, OutT *out, int64_t n) {
  __shared__ OutT sh[kScanThreads / 64 + 1];
  OutT carry = 0;
  for (int64_t b = 0; b < ntiles; b += kScanThreads) {
    const int64_t i = b + threadIdx.x;
    OutT v = i < ntiles ? tile_sum[i] : 0, total;
    OutT ex = block_exclusive_scan<OutT>(v, sh, total);
    if (i < ntiles) tile_sum[i] = ex + carry;
    carry += total;
  }
  if (threadIdx.x == 0) out[n] = carry;
}

template <typename OutT>
__global__ void k_scan_add(OutT *out, int64_t n, const OutT *tile_sum) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += tile_sum[i / kScanTile];
}

// rank_t[t]: the place the locate kernels' count took for the molecule inside its cell (any order; the
// cells are sorted by molecule id next).
__global__ void k_scatter(const int32_t *cell_t, const int32_t *trav, int64_t n, const int32_t *cell_start,
                          const int32_t *rank_t, int32_t *perm) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int32_t c = cell_t[t];
  if (c >= 0) perm[cell_start[c] + rank_t[t]] = trav ? trav[t] : (int32_t)t;  // c < 0: unlocated (an error)
}

// Ascending molecule id inside every cell (the scatter's atomics leave an arbitrary order).
__global__ void k_sort_cells(const int32_t *cell_start, int64_t nc, int32_t *perm) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const int32_t b = cell_start[c], e = cell_start[c + 1];
  for (int32_t i = b + 1; i < e; ++i) {
    const int32_t v = perm[i];
    int32_t j = i - 1;
    while (j >= b && perm[j] > v) {
      perm[j + 1] = perm[j];
      --j;
    }
    perm[j + 1] = v;
  }
}

__global__ void k_group_ranges(const int32_t *cell_start, const int32_t *g_cell0, int64_t ng, int32_t *g_start,
                               int32_t *mol_group) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a > ng) return;
  const int32_t s = cell_start[g_cell0[a]];
  g_start[a] = s;
  if (a < ng) {
    const int32_t e = cell_start[g_cell0[a + 1]];
    for (int32_t m = s; m < e; ++m) mol_group[m] = (int32_t)a;
  }
}

__global__ void k_entry_counts(const int32_t *e_B, int64_t E, const int32_t *g_start, int32_t *cnt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int32_t B = e_B[e];
  cnt[e] = g_start[B + 1] - g_start[B];
}

template <typename T>
__global__ void k_fill(T *p, int64_t n, T v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// =====================================================================================================
// kernels: forces

template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  using type = float4;
};
template <>
struct Vec4<double> {
  using type = double4;
};

// Gather positions into cell-sorted order, in group-local coordinates (x - origin of the molecule's
// group); the species id rides in .w as integer bits.
template <typename T, typename PT>
__global__ void k_gather(const PT *__restrict__ pos, const int32_t *__restrict__ species, const int32_t *perm,
                         const int32_t *mol_group, const double *orig, int64_t n, int nsp,
                         typename Vec4<T>::type *out) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  const int32_t id = perm[m];
  const int32_t a = mol_group[m];
  typename Vec4<T>::type v;
  v.x = (T)((double)pos[3 * (int64_t)id] - orig[3 * (int64_t)a]);
  v.y = (T)((double)pos[3 * (int64_t)id + 1] - orig[3 * (int64_t)a + 1]);
  v.z = (T)((double)pos[3 * (int64_t)id + 2] - orig[3 * (int64_t)a + 2]);
  const int32_t t = species ? min(max(species[id], 0), nsp - 1) : 0;  // out-of-range ids are clamped
  if constexpr (sizeof(T) == 4)
    v.w = __builtin_bit_cast(float, t);
  else
    v.w = __builtin_bit_cast(double, (int64_t)t);
  out[m] = v;
}

struct LJTab {
  float sig2[64], e24[64], e4[64];
  double sig2d[64], e24d[64], e4d[64];
  float rc2, band;
  float rc2lo, rc2hi;  // rc^2 -+ band: an FP32 s below rc2lo is surely inside, at or above rc2hi surely outside
  double rc2d;
  int nsp;
};

template <typename T>
__device__ __forceinline__ int type_of(T w) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(int, w);
  else
    return (int)__builtin_bit_cast(int64_t, w);
}

template <typename T>
__device__ __forceinline__ T tab_sig2(const LJTab &t, int k) {
  if constexpr (sizeof(T) == 4) return t.sig2[k]; else return t.sig2d[k];
}
template <typename T>
__device__ __forceinline__ T tab_e24(const LJTab &t, int k) {
  if constexpr (sizeof(T) == 4) return t.e24[k]; else return t.e24d[k];
}
template <typename T>
__device__ __forceinline__ T tab_e4(const LJTab &t, int k) {
  if constexpr (sizeof(T) == 4) return t.e4[k]; else return t.e4d[k];
}

// Per-lane Lennard-Jones parameters of the lane's i-species against j-species 0 and 1 (MIX <= 1),
// or the full table (MIX == 2: looked up per pair).
template <typename T, int MIX>
struct LaneLJ {
  T s0, s1, g0, g1, u0, u1;
  int ti;
  // One or two species: the parameters are selected from kernel-argument values (no per-lane
  // memory access, which would otherwise be waited for inside the pair loops).
  __device__ __forceinline__ void init(const LJTab &t, int ti_) {
    ti = ti_;
    if (MIX == 0) {
      s0 = tab_sig2<T>(t, 0);
      g0 = tab_e24<T>(t, 0);
      u0 = tab_e4<T>(t, 0);
    } else if (MIX == 1) {
      const bool b = ti != 0;
      s0 = b ? tab_sig2<T>(t, 8) : tab_sig2<T>(t, 0);
      g0 = b ? tab_e24<T>(t, 8) : tab_e24<T>(t, 0);
      u0 = b ? tab_e4<T>(t, 8) : tab_e4<T>(t, 0);
      s1 = b ? tab_sig2<T>(t, 9) : tab_sig2<T>(t, 1);
      g1 = b ? tab_e24<T>(t, 9) : tab_e24<T>(t, 1);
      u1 = b ? tab_e4<T>(t, 9) : tab_e4<T>(t, 1);
    } else {
      s0 = tab_sig2<T>(t, ti * 8);
      g0 = tab_e24<T>(t, ti * 8);
      u0 = tab_e4<T>(t, ti * 8);
    }
  }
  __device__ __forceinline__ void get(const LJTab &t, int tj, T &sig2, T &e24, T &e4) const {
    if (MIX == 0) {
      sig2 = s0;
      e24 = g0;
      e4 = u0;
    } else if (MIX == 1) {
      const bool b = tj != 0;
      sig2 = b ? s1 : s0;
      e24 = b ? g1 : g0;
      e4 = b ? u1 : u0;
    } else {
      const int k = ti * 8 + tj;
      sig2 = tab_sig2<T>(t, k);
      e24 = tab_e24<T>(t, k);
      e4 = tab_e4<T>(t, k);
    }
  }
};

__device__ __forceinline__ float fast_rcp(float s) { return __builtin_amdgcn_rcpf(s); }
// FP64: the hardware reciprocal refined by two Newton steps (about 1 ulp, against the ten instructions of
// a correctly rounded division; the FP64 path's bar is 1e-12 of the result)
__device__ __forceinline__ double fast_rcp(double s) {
  double r = __builtin_amdgcn_rcp(s);
  r = fma(r, fma(-s, r, 1.0), r);
  return fma(r, fma(-s, r, 1.0), r);
}

template <typename T>
__device__ __forceinline__ T far_i() { return (T)1e15; }
template <typename T>
__device__ __forceinline__ T far_j() { return (T)-1e15; }

}  // namespace

#include "aica_pair.inc"
#include "aica_adjoint_pair.inc"

namespace {

// Deterministic two-stage reduction of per-group partials.  Stage 1: block b sums the fixed row range
// [b * chunk, (b + 1) * chunk) of a row-major [ng][stride] array (columns col0 .. col0 + K - 1, doubles or
// unsigned integers read as doubles; integer sums stay exact below 2^53) in a fixed thread order and
// tree.  Stage 2 (one block) sums the stage-1 rows in block order.
constexpr int kRedBlocks = 512, kRedThreads = 256;

template <int K, typename S>
__global__ __launch_bounds__(kRedThreads) void k_reduce_rows(const S *in, int64_t ng, int stride, int col0,
                                                              int64_t chunk, double *part) {
  __shared__ double sh[K][kRedThreads];
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0;
  const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = std::min<int64_t>(ng, r0 + chunk);
  for (int64_t r = r0 + threadIdx.x; r < r1; r += kRedThreads)
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += (double)in[(int64_t)stride * r + col0 + k];
#pragma unroll
  for (int k = 0; k < K; ++k) sh[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int o = kRedThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
#pragma unroll
      for (int k = 0; k < K; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) part[(int64_t)K * blockIdx.x + k] = sh[k][0];
}

// Stage 2 helper: thread 0 ends with the column sums of part[nb][K] in out[K].
template <int K>
__device__ void reduce_part_rows(const double *part, int nb, double *out) {
  __shared__ double sh[K][kRedThreads];
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0;
  for (int b = threadIdx.x; b < nb; b += kRedThreads)
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] += part[(int64_t)K * b + k];
#pragma unroll
  for (int k = 0; k < K; ++k) sh[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int o = kRedThreads / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
#pragma unroll
      for (int k = 0; k < K; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = sh[k][0];
}

// U, W (FP64) and the pair count from the stage-1 rows (U, W) and (npairs).
__global__ __launch_bounds__(kRedThreads) void k_reduce_uw(const double *part_uw, const double *part_np, int nb,
                                                            double *uw, int64_t *npairs) {
  double a[2], c[1];
  reduce_part_rows<2>(part_uw, nb, a);
  __syncthreads();
  reduce_part_rows<1>(part_np, nb, c);
  if (threadIdx.x == 0) {
    if (uw) {
      uw[0] = a[0];
      uw[1] = a[1];
    }
    if (npairs) npairs[0] = (int64_t)c[0];
  }
}

inline int red_blocks(int64_t ng, int64_t &chunk) {
  const int nb = (int)std::min<int64_t>(kRedBlocks, std::max<int64_t>(1, (ng + kRedThreads - 1) / kRedThreads));
  chunk = (std::max<int64_t>(ng, 1) + nb - 1) / nb;
  return nb;
}

inline unsigned grid1d(int64_t n, int b) { return (unsigned)std::max<int64_t>(1, (n + b - 1) / b); }

template <typename OutT>
int scan_exclusive(aica_dil *h, const int32_t *in, int64_t n, OutT *out, hipStream_t st) {
  const int64_t ntiles = std::max<int64_t>(1, (n + kScanTile - 1) / kScanTile);
  int rc = h->d_scan_tmp.ensure(sizeof(OutT) * (ntiles + 1));
  if (rc) return rc;
  OutT *ts = h->d_scan_tmp.as<OutT>();
  hipLaunchKernelGGL((k_scan_tiles<int32_t, OutT>), dim3((unsigned)ntiles), dim3(kScanThreads), 0, st, in, n, out, ts);
  hipLaunchKernelGGL((k_scan_sums<OutT>), dim3(1), dim3(kScanThreads), 0, st, ts, ntiles, out, n);
  hipLaunchKernelGGL((k_scan_add<OutT>), dim3(grid1d(n, 256)), dim3(256), 0, st, out, n, (const OutT *)ts);
  HIPCHK(hipGetLastError());
  return AICA_OK;
}

struct ProfScope {
  aica_dil *h;
  const char *name;
  hipStream_t st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ProfScope(aica_dil *h_, const char *n, hipStream_t s) : h(h_), name(n), st(s) {
    if (h->profiling) {
      (void)hipEventCreate(&e0);
      (void)hipEventCreate(&e1);
      (void)hipEventRecord(e0, st);
    }
  }
  ~ProfScope() {
    if (h->profiling && e0) {
      (void)hipEventRecord(e1, st);
      h->timers[name].pending.push_back({e0, e1});
      h->timers[name].launches++;
    }
  }
};

}  // namespace

// =====================================================================================================
// setup helpers

static int upload_geometry(aica_dil *h) {
  const Geometry &g = h->geo;
  int rc;
  // cell records for point location, in sorted cell order (layout described at point_in_rec)
  {
    std::vector<int64_t> roff(g.nc + 1, 0);
    for (int64_t s = 0; s < g.nc; ++s) {
      const int64_t c = h->order[s];
      int64_t sz = 4;
      for (int64_t k = g.cf_off[c]; k < g.cf_off[c + 1]; ++k) {
        const int32_t f = g.cf[k];
        sz += 4 + 3 * (g.foff[f + 1] - g.foff[f]);
      }
      roff[s + 1] = roff[s] + sz;
    }
    std::vector<double> rec(roff[g.nc]);
    parallel_for(g.nc, [&](int64_t s0, int64_t s1, int) {
      for (int64_t s = s0; s < s1; ++s) {
        const int64_t c = h->order[s];
        const int64_t nf = g.cf_off[c + 1] - g.cf_off[c];
        double *R = rec.data() + roff[s];
        R[0] = (double)nf;
        for (int q = 0; q < 3; ++q) R[1 + q] = g.ccen[3 * c + q];
        double *FC = R + 4, *LEN = FC + 3 * nf, *V = LEN + nf;
        for (int64_t k = 0; k < nf; ++k) {
          const int32_t f = g.cf[g.cf_off[c] + k];
          const int64_t b0 = g.foff[f], len = g.foff[f + 1] - b0;
          const bool rev = g.cf_sgn[g.cf_off[c] + k] < 0;  // the neighbour side walks the loop backwards
          for (int q = 0; q < 3; ++q) FC[3 * k + q] = g.fcen[3 * (int64_t)f + q];
          LEN[k] = (double)len;
          for (int64_t j = 0; j < len; ++j) {
            const int64_t jj = rev ? (len - j) % len : j;
            for (int q = 0; q < 3; ++q) V[3 * j + q] = g.pts[3 * (int64_t)g.fpts[b0 + jj] + q];
          }
          V += 3 * len;
        }
      }
    });
    if ((rc = upload(h->d_rec_off, roff))) return rc;
    if ((rc = upload(h->d_rec, rec))) return rc;
    // FP32 records (layout at surely_in_rec32), when every cell fits the fixed stride
    bool fits = true;
    for (int64_t s = 0; s < g.nc && fits; ++s) {
      const double *R = rec.data() + roff[s];
      const int64_t nf = (int64_t)R[0];
      int64_t nv = 0;
      for (int64_t k = 0; k < nf; ++k) nv += (int64_t)R[4 + 3 * nf + k];
      fits = 2 + nf + nv <= kR32;
    }
    h->has_rec32 = fits;
    if (fits) {
      std::vector<float4> r32((size_t)g.nc * kR32), pl32((size_t)g.nc * kPl);
      parallel_for(g.nc, [&](int64_t s0, int64_t s1, int) {
        for (int64_t s = s0; s < s1; ++s) {
          const double *R = rec.data() + roff[s];
          const int64_t nf = (int64_t)R[0];
          float4 *O = r32.data() + (size_t)s * kR32;
          const double a[3] = {(double)(float)R[1], (double)(float)R[2], (double)(float)R[3]};
          const double *FC = R + 4, *LEN = FC + 3 * nf, *V = LEN + nf;
          // the cell's size: the largest distance from the vertex mean to a face centroid
          double size = 0;
          for (int64_t k = 0; k < nf; ++k) {
            const double e0 = FC[3 * k] - R[1], e1 = FC[3 * k + 1] - R[2], e2 = FC[3 * k + 2] - R[3];
            size = std::max(size, std::sqrt(e0 * e0 + e1 * e1 + e2 * e2));
          }
          O[0] = make_float4((float)nf, (float)a[0], (float)a[1], (float)a[2]);
          O[1] = make_float4((float)(R[1] - a[0]), (float)(R[2] - a[1]), (float)(R[3] - a[2]), (float)size);
          // plane records (layout at plane_ball): the face loops run with the right-hand normal out of the cell
          float4 *PL = pl32.data() + (size_t)s * kPl;
          for (int k = 0; k < kPl; ++k) PL[k] = make_float4(0.f, 0.f, 0.f, -3.0e38f);
          {
            int ntri = 0;
            const double *Vk = V;
            for (int64_t k = 0; k < nf; ++k) {
              const int64_t len = (int64_t)LEN[k];
              const double *f = FC + 3 * k;
              for (int64_t j = 0; j < len; ++j) {
                const double *v0 = Vk + 3 * j, *v1 = Vk + 3 * ((j + 1) % len);
                const double u[3] = {v0[0] - f[0], v0[1] - f[1], v0[2] - f[2]};
                const double w[3] = {v1[0] - f[0], v1[1] - f[1], v1[2] - f[2]};
                double nrm[3] = {-(u[1] * w[2] - u[2] * w[1]), -(u[2] * w[0] - u[0] * w[2]), -(u[0] * w[1] - u[1] * w[0])};
                const double nn = std::sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
                if (ntri < kPl && nn > 0) {
                  for (int q = 0; q < 3; ++q) nrm[q] /= nn;
                  const double dd = nrm[0] * (f[0] - a[0]) + nrm[1] * (f[1] - a[1]) + nrm[2] * (f[2] - a[2]);
                  PL[ntri] = make_float4((float)nrm[0], (float)nrm[1], (float)nrm[2], (float)dd);
                }
                if (!(nn > 0)) ntri = kPl;  // a degenerate triangle: no plane test for this cell
                ++ntri;
              }
              Vk += 3 * len;
            }
            if (ntri > kPl) PL[0] = make_float4(0.f, 0.f, 0.f, 3.0e38f);
          }
          int64_t nv = 0;
          for (int64_t k = 0; k < nf; ++k) {
            O[2 + k] = make_float4((float)(FC[3 * k] - a[0]), (float)(FC[3 * k + 1] - a[1]), (float)(FC[3 * k + 2] - a[2]),
                                   (float)LEN[k]);
            nv += (int64_t)LEN[k];
          }
          for (int64_t j = 0; j < nv; ++j)
            O[2 + nf + j] = make_float4((float)(V[3 * j] - a[0]), (float)(V[3 * j + 1] - a[1]), (float)(V[3 * j + 2] - a[2]), 0.f);
          // the cell across each face, on the first vertex of the face's loop
          const int64_t c = h->order[s];
          int64_t v0 = 0;
          for (int64_t k = 0; k < nf; ++k) {
            const int32_t f = g.cf[g.cf_off[c] + k];
            const int64_t other = g.own[f] == c ? g.nei[f] : g.own[f];
            const int32_t across = g.nei[f] >= 0 && other >= 0 ? (int32_t)h->rank[other] : -1;
            O[2 + nf + v0].w = __builtin_bit_cast(float, across);
            v0 += (int64_t)LEN[k];
          }
        }
      });
      if ((rc = upload(h->d_rec32, r32))) return rc;
      if ((rc = upload(h->d_pl32, pl32))) return rc;
    }
  }
  // cells across each cell's interior faces, sorted ids in sorted cell order
  {
    std::vector<int64_t> noff(g.nc + 1, 0);
    const int64_t nf = g.nf;
    for (int64_t f = 0; f < nf; ++f)
      if (g.nei[f] >= 0) {
        noff[h->rank[g.own[f]] + 1]++;
        noff[h->rank[g.nei[f]] + 1]++;
      }
    for (int64_t s = 0; s < g.nc; ++s) noff[s + 1] += noff[s];
    std::vector<int32_t> nb(noff[g.nc]);
    std::vector<int64_t> fill(noff.begin(), noff.end() - 1);
    for (int64_t f = 0; f < nf; ++f)
      if (g.nei[f] >= 0) {
        const int32_t a = h->rank[g.own[f]], b = h->rank[g.nei[f]];
        nb[fill[a]++] = b;
        nb[fill[b]++] = a;
      }
    if ((rc = upload(h->d_nbr_off, noff))) return rc;
    if ((rc = upload(h->d_nbr, nb))) return rc;
  }
  // padded bounding boxes (sorted cell order) and the point-location grid (sorted cell indices listed in
  // every bin their box touches, in ascending mesh cell id so the lowest containing cell is found first)
  std::vector<double> bb(6 * g.nc);
  for (int64_t c = 0; c < g.nc; ++c)
    for (int q = 0; q < 3; ++q) {
      const double ext = g.hi[3 * c + q] - g.lo[3 * c + q];
      bb[6 * c + q] = g.lo[3 * c + q] - 1e-9 * ext;
      bb[6 * c + 3 + q] = g.hi[3 * c + q] + 1e-9 * ext;
    }
  {
    std::vector<double> bbs(6 * g.nc);
    for (int64_t s = 0; s < g.nc; ++s)
      for (int q = 0; q < 6; ++q) bbs[6 * s + q] = bb[6 * (int64_t)h->order[s] + q];
    if ((rc = upload(h->d_bb, bbs))) return rc;
  }
  double gh = std::cbrt(g.total_volume / (double)g.nc);
  for (int q = 0; q < 3; ++q) gh = std::max(gh, (g.dom_hi[q] - g.dom_lo[q]) / 2048.0);
  int64_t nb[3];
  for (int q = 0; q < 3; ++q) {
    h->glo[q] = g.dom_lo[q] - 1e-9 * (g.dom_hi[q] - g.dom_lo[q]) - 1e-300;
    nb[q] = std::max<int64_t>(1, (int64_t)std::ceil((g.dom_hi[q] + 1e-9 * (g.dom_hi[q] - g.dom_lo[q]) - h->glo[q]) / gh));
    h->gnb[q] = nb[q];
  }
  h->gh = gh;
  const int64_t nbins = nb[0] * nb[1] * nb[2];
  std::vector<int64_t> off(nbins + 1, 0);
  auto range = [&](int64_t c, int q, int64_t &b0, int64_t &b1) {
    b0 = (int64_t)std::floor((bb[6 * c + q] - h->glo[q]) / gh);
    b1 = (int64_t)std::floor((bb[6 * c + 3 + q] - h->glo[q]) / gh);
    b0 = std::min(std::max<int64_t>(b0, 0), nb[q] - 1);
    b1 = std::min(std::max<int64_t>(b1, 0), nb[q] - 1);
  };
  for (int64_t c = 0; c < g.nc; ++c) {
    int64_t lo[3], hi[3];
    for (int q = 0; q < 3; ++q) range(c, q, lo[q], hi[q]);
    for (int64_t z = lo[2]; z <= hi[2]; ++z)
      for (int64_t y = lo[1]; y <= hi[1]; ++y)
        for (int64_t x = lo[0]; x <= hi[0]; ++x) off[x + nb[0] * (y + nb[1] * z) + 1]++;
  }
  for (int64_t b = 0; b < nbins; ++b) off[b + 1] += off[b];
  std::vector<int32_t> cells(off[nbins]);
  std::vector<int64_t> fill(off.begin(), off.end() - 1);
  for (int64_t c = 0; c < g.nc; ++c) {
    int64_t lo[3], hi[3];
    for (int q = 0; q < 3; ++q) range(c, q, lo[q], hi[q]);
    for (int64_t z = lo[2]; z <= hi[2]; ++z)
      for (int64_t y = lo[1]; y <= hi[1]; ++y)
        for (int64_t x = lo[0]; x <= hi[0]; ++x) cells[fill[x + nb[0] * (y + nb[1] * z)]++] = h->rank[c];
  }
  if ((rc = upload(h->d_gb_off, off))) return rc;
  if ((rc = upload(h->d_gb_cell, cells))) return rc;
  return AICA_OK;
}

static int ensure_groups(aica_dil *h, int64_t n) {
  if (h->groups_ready && h->groups_for_n == n) return AICA_OK;
  auto t0 = std::chrono::steady_clock::now();
  const double density = (double)n / h->geo.total_volume;
  double target = 64.0;  // largest expected occupancy of a group (k-d subtree; measured best on the channel)
  if (const char *e = getenv("AICA_GROUP_TARGET")) target = std::max(1.0, atof(e));
  int rc = build_groups(h->geo, h->order, h->split_depth, h->pairs, density, target, h->grp);
  if (rc) return rc;
  const Groups &G = h->grp;
  const int64_t E = G.e_off[G.ng];
  std::vector<float4> v32(E);
  std::vector<double4> v64(E);
  // Entry offsets: a j of group B at xm relative to orig_B is referred into A's frame at R xm + o with
  // o = T(orig_B) - orig_A (R = I and o = orig_B + t - orig_A for a translation).  The fourth component
  // holds the image code, plus kRotFlag when the image has a rotation (whose R the kernels look up).
  for (int64_t e = 0; e < E; ++e) {
    const int64_t B = G.e_B[e];
    int64_t A = std::upper_bound(G.e_off.begin(), G.e_off.end(), e) - G.e_off.begin() - 1;
    const Xf T = image_transform(h->geo, G.e_img[3 * e], G.e_img[3 * e + 1], G.e_img[3 * e + 2]);
    double o[3];
    if (T.rot) {
      double tb[3];
      T.apply(&G.orig[3 * B], tb);
      for (int q = 0; q < 3; ++q) o[q] = tb[q] - G.orig[3 * A + q];
    } else {
      for (int q = 0; q < 3; ++q) o[q] = G.orig[3 * B + q] + T.y[q] - G.orig[3 * A + q];
    }
    const int code = 9 * (G.e_img[3 * e] + 1) + 3 * (G.e_img[3 * e + 1] + 1) + (G.e_img[3 * e + 2] + 1) +
                     (T.rot ? kRotFlag : 0);
    v32[e] = make_float4((float)o[0], (float)o[1], (float)o[2], __builtin_bit_cast(float, code));
    v64[e] = make_double4(o[0], o[1], o[2], __builtin_bit_cast(double, (int64_t)code));
  }
  if (h->geo.has_rot) {  // R of every image code (the identity for translations)
    std::vector<double> r64(27 * 9);
    for (int code = 0; code < 27; ++code) {
      const Xf T = image_transform(h->geo, code / 9 - 1, (code / 3) % 3 - 1, code % 3 - 1);
      for (int i = 0; i < 9; ++i) {
        r64[9 * code + i] = T.R[i];
      }
    }
    if ((rc = upload(h->d_rot64, r64))) return rc;
  }
  if ((rc = upload(h->d_g_cell0, G.cell0))) return rc;
  if ((rc = upload(h->d_e_off, G.e_off))) return rc;
  if ((rc = upload(h->d_e_B, G.e_B))) return rc;
  if ((rc = upload(h->d_e_vec32, v32))) return rc;
  if ((rc = upload(h->d_e_vec64, v64))) return rc;
  if ((rc = upload(h->d_nl_off, G.nl_off))) return rc;
  if ((rc = upload(h->d_nl_e, G.nl_e))) return rc;
  if ((rc = upload(h->d_nl_d, G.nl_d))) return rc;
  if ((rc = upload(h->d_nl_r, G.nl_r))) return rc;
  {
    std::vector<int32_t> rcnt(h->geo.nc);
    for (int64_t d = 0; d < h->geo.nc; ++d) rcnt[d] = (int32_t)(G.rc_off[d + 1] - G.rc_off[d] + 1);
    if ((rc = upload(h->d_rcnt, rcnt))) return rc;
  }
  if ((rc = upload(h->d_orig, G.orig))) return rc;
  h->groups_ready = true;
  h->groups_for_n = n;
  h->group_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return AICA_OK;
}

// =====================================================================================================
// C ABI (every entry point is declared extern "C" in aica.h)

const char *aica_last_error(void) { return last_error_cstr(); }

int aica_build_dil(const aica_mesh *mesh, double rcut, double guard, aica_dil **out) {
  return aica_build_dil_ex(mesh, rcut, guard, AICA_DIL_CLOSEST, out);
}

int aica_build_dil_ex(const aica_mesh *mesh, double rcut, double guard, int32_t predicate, aica_dil **out) {
  if (!out) return fail(AICA_E_INVAL, "out is NULL");
  *out = nullptr;
  if (predicate != AICA_DIL_CLOSEST && predicate != AICA_DIL_VERTEX)
    return fail(AICA_E_INVAL, "predicate must be AICA_DIL_CLOSEST or AICA_DIL_VERTEX");
  if (!(rcut > 0) || !std::isfinite(rcut) || !(guard >= 0) || !std::isfinite(guard))
    return fail(AICA_E_INVAL, "rcut must be > 0 and guard >= 0");
  auto t0 = std::chrono::steady_clock::now();
  aica_dil *h = new (std::nothrow) aica_dil();
  if (!h) return fail(AICA_E_NOMEM, "handle allocation failed");
  int rc = build_geometry(mesh, h->geo);
  if (rc) {
    delete h;
    return rc;
  }
  h->rcut = rcut;
  h->guard = guard;
  const bool verbose = getenv("AICA_VERBOSE") != nullptr;
  auto t1 = std::chrono::steady_clock::now();
  spatial_order(h->geo, h->order, h->rank, h->split_depth);
  auto t2 = std::chrono::steady_clock::now();
  rc = build_cell_pairs(h->geo, h->order, h->rank, rcut + guard, predicate, h->pairs);
  if (verbose)
    fprintf(stderr, "aica_build_dil: geometry %.2fs order %.2fs pairs %.2fs (%zu)\n",
            std::chrono::duration<double>(t1 - t0).count(), std::chrono::duration<double>(t2 - t1).count(),
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t2).count(), h->pairs.size());
  if (rc) {
    delete h;
    return rc;
  }
  h->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  *out = h;
  return AICA_OK;
}

void aica_dil_free(aica_dil *h) {
  if (!h) return;
  for (auto &kv : h->timers)
    for (auto &ev : kv.second.pending) {
      (void)hipEventDestroy(ev.first);
      (void)hipEventDestroy(ev.second);
    }
  delete h;
}

int aica_bin(aica_dil *h, const void *pos_dev, int32_t pos_dtype, int64_t n, void *hip_stream) {
  if (!h) return fail(AICA_E_INVAL, "handle is NULL");
  h->bin_valid = false;
  h->wsteps_valid = false;
  if (n < 0 || (n > 0 && !pos_dev)) return fail(AICA_E_INVAL, "bad positions");
  if (n >= (1LL << 28) - 1) return fail(AICA_E_INVAL, "too many molecules (the pair kernels take fewer than 2^28 - 1)");
  if (pos_dtype != AICA_FP32 && pos_dtype != AICA_FP64) return fail(AICA_E_INVAL, "pos_dtype must be AICA_FP32 or AICA_FP64");
  hipStream_t st = (hipStream_t)hip_stream;
  int rc;
  if (!h->geometry_on_device) {
    // the device copy of the geometry is made on first use, so that setup and the interaction
    // lists can be built and inspected without a GPU
    if (hipGetDevice(&h->device) != hipSuccess) return fail(AICA_E_HIP, "no HIP device");
    if ((rc = upload_geometry(h))) return rc;
    h->geometry_on_device = true;
  }
  rc = ensure_groups(h, n);
  if (rc) return rc;
  const int64_t nc = h->geo.nc, ng = h->grp.ng, E = h->grp.e_off[ng];
  if ((rc = h->d_cell_of.ensure(4 * std::max<int64_t>(n, 1)))) return rc;
  if ((rc = h->d_count.ensure(4 * nc))) return rc;
  if ((rc = h->d_cell_start.ensure(4 * (nc + 1)))) return rc;
  if ((rc = h->d_rank.ensure(4 * std::max<int64_t>(n, 1)))) return rc;
  if ((rc = h->d_perm.ensure(4 * std::max<int64_t>(n, 1)))) return rc;
  if ((rc = h->d_g_start.ensure(4 * (ng + 1)))) return rc;
  if ((rc = h->d_mol_group.ensure(4 * std::max<int64_t>(n, 1)))) return rc;
  if ((rc = h->d_jcnt.ensure(4 * std::max<int64_t>(nc, 1)))) return rc;
  if ((rc = h->d_slot_base.ensure(8 * (nc + 1)))) return rc;
  if ((rc = h->d_cell_sorted.ensure(4 * std::max<int64_t>(n, 1)))) return rc;
  if ((rc = h->d_status.ensure(8 * (8 + kRouteSlots)))) return rc;
  if ((rc = h->d_slow.ensure(4 * std::max<int64_t>(n, 1)))) return rc;
  if ((rc = h->d_ref.ensure(16 * std::max<int64_t>(n, 1)))) return rc;

  ProfScope ps(h, "bin", st);
  unsigned long long *status = h->d_status.as<unsigned long long>();
  // status: [0] unlocated, [1] over-full cells, [2] slow-kernel molecules, [8 ..) counters of the molecules
  // the records located
  hipLaunchKernelGGL((k_fill<unsigned long long>), dim3(1), dim3(8 + kRouteSlots), 0, st, status,
                     (int64_t)(8 + kRouteSlots), 0ull);
  unsigned long long *routes = status + 8;
  hipLaunchKernelGGL((k_fill<int32_t>), dim3(grid1d(nc, 256)), dim3(256), 0, st, h->d_count.as<int32_t>(), nc, 0);
  // the previous binning of the same n (if any) gives the traversal order and the hints: its
  // permutation moves to d_perm_prev, and d_cell_sorted still holds its cells until rebuilt below
  const bool prev = h->perm_n == n && n > 0;
  h->perm_n = -1;
  if (prev) h->d_perm.swap(h->d_perm_prev);
  if ((rc = h->d_perm.ensure(4 * std::max<int64_t>(n, 1)))) return rc;
  const int32_t *trav = prev ? h->d_perm_prev.as<int32_t>() : nullptr;
  const int32_t *hint = prev ? h->d_cell_sorted.as<int32_t>() : nullptr;
  if (n > 0) {
    const float4 *r32 = h->has_rec32 ? h->d_rec32.as<float4>() : nullptr;
    const float4 *pl = h->has_rec32 ? h->d_pl32.as<float4>() : nullptr;
    int32_t *slow = h->d_slow.as<int32_t>();
    unsigned long long *nslow = status + 2;
    // lanes per molecule of the slow kernel: a whole wave, or 16 (four molecules per wave) when the previous
    // binning sent more molecules down the slow path than the grid below has waves
    const bool slow16 = prev && h->located[2] > 4 * 2048;
#define AICA_LOCATE(PT)                                                                                            \
  hipLaunchKernelGGL((k_locate_fast<PT>), dim3(grid1d(n, 256 * kLocPerLane)), dim3(256), 0, st, (const PT *)pos_dev, \
                     n, trav, hint, r32, pl, h->d_ref.as<float4>(), h->d_cell_of.as<int32_t>(), h->d_rank.as<int32_t>(), \
                     h->d_count.as<int32_t>(), nslow, slow, routes);                                               \
  hipLaunchKernelGGL(!prev ? (k_locate_slow<PT, 1>) : slow16 ? (k_locate_slow<PT, 16>) : (k_locate_slow<PT, 64>), \
                     dim3(std::min<int64_t>(prev ? grid1d(n, 4) : grid1d(n, 256), 2048)), dim3(256), 0, st,        \
                     (const PT *)pos_dev, nslow, slow, trav, hint, r32, pl, h->d_rec_off.as<int64_t>(),          \
                     h->d_rec.as<double>(), h->d_nbr_off.as<int64_t>(),                                            \
                     h->d_nbr.as<int32_t>(), h->d_bb.as<double>(), h->d_gb_off.as<int64_t>(),                       \
                     h->d_gb_cell.as<int32_t>(), h->glo[0], h->glo[1], h->glo[2], h->gh, h->gnb[0], h->gnb[1],      \
                     h->gnb[2], h->d_ref.as<float4>(), h->d_cell_of.as<int32_t>(), h->d_rank.as<int32_t>(),       \
                     h->d_count.as<int32_t>(), status)
    if (pos_dtype == AICA_FP64) {
      AICA_LOCATE(double);
    } else {
      AICA_LOCATE(float);
    }
#undef AICA_LOCATE
    HIPCHK(hipGetLastError());
  }
  // the unlocated count is read with the other counts below (one synchronisation per binning); an
  // unlocated molecule is left out of the occupancy and of the permutation
  if ((rc = scan_exclusive<int32_t>(h, h->d_count.as<int32_t>(), nc, h->d_cell_start.as<int32_t>(), st))) return rc;
  if (n > 0)
    hipLaunchKernelGGL(k_scatter, dim3(grid1d(n, 256)), dim3(256), 0, st, h->d_cell_of.as<int32_t>(), trav, n,
                       h->d_cell_start.as<int32_t>(), h->d_rank.as<int32_t>(), h->d_perm.as<int32_t>());
  hipLaunchKernelGGL(k_sort_cells, dim3(grid1d(nc, 256)), dim3(256), 0, st, h->d_cell_start.as<int32_t>(), nc,
                     h->d_perm.as<int32_t>());
  hipLaunchKernelGGL(k_group_ranges, dim3(grid1d(ng + 1, 256)), dim3(256), 0, st, h->d_cell_start.as<int32_t>(),
                     h->d_g_cell0.as<int32_t>(), ng, h->d_g_start.as<int32_t>(), h->d_mol_group.as<int32_t>());
  hipLaunchKernelGGL(k_slot_counts, dim3(grid1d(nc, 256)), dim3(256), 0, st, h->d_count.as<int32_t>(),
                     h->d_rcnt.as<int32_t>(), nc, h->d_jcnt.as<int32_t>());
  hipLaunchKernelGGL(k_cell_of_sorted, dim3(grid1d(nc, 256)), dim3(256), 0, st, h->d_cell_start.as<int32_t>(), nc,
                     h->d_cell_sorted.as<int32_t>());
  HIPCHK(hipGetLastError());
  if ((rc = scan_exclusive<int64_t>(h, h->d_jcnt.as<int32_t>(), nc, h->d_slot_base.as<int64_t>(), st))) return rc;
  int64_t jt = 0;
  unsigned long long stat[8 + kRouteSlots];
  HIPCHK(hipMemcpyAsync(&jt, h->d_slot_base.as<int64_t>() + nc, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(stat, status, sizeof stat, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const unsigned long long unl = stat[0];
  if (unl > 0) return fail(AICA_E_UNLOCATED, std::to_string(unl) + " molecule(s) lie in no mesh cell");
  h->located[1] = 0;
  for (int k = 0; k < kRouteSlots; ++k) h->located[1] += (int64_t)stat[8 + k];
  h->located[2] = (int64_t)stat[2];
  h->located[0] = n - h->located[1] - h->located[2];
  if (jt >= (1LL << 31)) return fail(AICA_E_NOMEM, "reaction slots exceed 2^31; split the system");
  h->perm_n = n;  // d_perm holds this binning's permutation
  h->jtotal = jt;
  h->n = n;
  h->bin_pos = pos_dev;
  h->bin_dtype = pos_dtype;
  h->bin_valid = true;
  return AICA_OK;
}

static int build_tab(const aica_dil *h, const aica_params *p, LJTab &t) {
  if (!p) return fail(AICA_E_INVAL, "params is NULL");
  if (!(p->rcut > 0) || p->rcut > h->rcut * (1 + 1e-15))
    return fail(AICA_E_INVAL, "params.rcut must be > 0 and not exceed the DIL's rcut");
  if (p->n_species < 1 || p->n_species > 8 || !p->eps || !p->sigma)
    return fail(AICA_E_INVAL, "n_species must be 1..8 with eps and sigma given");
  if (p->precision != AICA_FP32 && p->precision != AICA_FP64) return fail(AICA_E_INVAL, "bad precision");
  memset(&t, 0, sizeof t);
  for (int a = 0; a < p->n_species; ++a)
    if (!(p->eps[a] > 0) || !(p->sigma[a] > 0)) return fail(AICA_E_INVAL, "eps and sigma must be positive");
  for (int a = 0; a < p->n_species; ++a)
    for (int b = 0; b < p->n_species; ++b) {
      const double e = a == b ? p->eps[a] : std::sqrt(p->eps[a] * p->eps[b]);
      const double s = a == b ? p->sigma[a] : 0.5 * (p->sigma[a] + p->sigma[b]);
      const int k = a * 8 + b;
      t.sig2d[k] = s * s;
      t.e24d[k] = 24.0 * e;
      t.e4d[k] = 4.0 * e;
      t.sig2[k] = (float)(s * s);
      t.e24[k] = (float)(24.0 * e);
      t.e4[k] = (float)(4.0 * e);
    }
  t.rc2d = p->rcut * p->rcut;
  t.rc2 = (float)t.rc2d;
  t.band = (float)(t.rc2d * std::ldexp(1.0, -20));
  t.rc2lo = (float)(t.rc2d - (double)t.band);
  t.rc2hi = (float)(t.rc2d + (double)t.band);
  t.nsp = p->n_species;
  return AICA_OK;
}

// Device buffers of one force call: the handle's grow-only workspace, or regions of the fixed scratch array
// (aica_forces_noalloc).  pos: [n] gathered positions; own: [2n] (hi, lo) own records; jpart: [J] reaction
// records tagged with epoch; gpart, gnp: per-group partials; red: stage-1 reduction rows.
struct ForceWs {
  void *pos = nullptr, *own = nullptr, *jpart = nullptr, *gpart = nullptr, *gnp = nullptr, *red = nullptr;
  uint32_t epoch = 0;
};

// Reaction buffer: (re)allocate, fill with a pattern no epoch can equal, and advance the epoch.
static int prepare_jpart(aica_dil *h, size_t bytes, hipStream_t st) {
  const void *old = h->d_jpart.p;
  // a growing buffer gets 1/8 headroom: the slot count follows the occupancy of every step, and each
  // reallocation costs a fill of the whole buffer
  int rc = h->d_jpart.ensure(bytes > h->d_jpart.bytes ? bytes + bytes / 8 : bytes);
  if (rc) return rc;
  if (h->d_jpart.p != old || h->jpart_tagged < h->d_jpart.bytes || h->epoch >= kMaxEpoch) {
    const int64_t words = (int64_t)(h->d_jpart.bytes / 4);
    hipLaunchKernelGGL((k_fill<uint32_t>), dim3(grid1d(words, 256)), dim3(256), 0, st, h->d_jpart.as<uint32_t>(),
                       words, 0xFFFFFFFFu);
    HIPCHK(hipGetLastError());
    h->jpart_tagged = h->d_jpart.bytes;
    h->epoch = 0;
  }
  h->epoch += 1;
  return AICA_OK;
}

template <typename T, int MODE>
static int launch_pair(aica_dil *h, const ForceWs &ws, const LJTab &tab, bool comp, hipStream_t st, int64_t cap,
                       unsigned long long *pcount, int32_t *mol_count = nullptr) {
  using V4 = typename Vec4<T>::type;
  const int64_t ng = h->grp.ng;
  constexpr int NW = pair_waves(sizeof(T));
  const int64_t nblocks = (ng + NW - 1) / NW;
  const int64_t padded = ((nblocks + 7) / 8) * 8;
  const V4 *pos = (const V4 *)ws.pos;
  const V4 *ev = sizeof(T) == 4 ? (const V4 *)h->d_e_vec32.p : (const V4 *)h->d_e_vec64.p;
  T *jpart = MODE == 1 ? nullptr : (T *)ws.jpart;
  T *own = MODE == 1 ? nullptr : (T *)ws.own;
  double *gpart = MODE == 0 ? (double *)ws.gpart : nullptr;
  unsigned long long *gnp = MODE == 0 ? (unsigned long long *)ws.gnp : nullptr;
  int32_t *pairs_out = (MODE == 1 && cap >= 0) ? h->d_pairs.as<int32_t>() : nullptr;  // cap < 0: counts only
  // rotating referral: FP64 rotations and offsets for both precisions (the referred position is rounded once)
  const double *rot = h->geo.has_rot ? h->d_rot64.as<double>() : nullptr;
  const double4 *evd = h->geo.has_rot ? h->d_e_vec64.as<double4>() : nullptr;
  const int nsp = tab.nsp;
#define AICA_LAUNCH_R(MIX, COMP, ROT)                                                                              \
  hipLaunchKernelGGL((k_pair<T, MIX, MODE, COMP, ROT>), dim3((unsigned)padded), dim3(64 * NW), 0, st, pos,         \
                     h->d_g_start.as<int32_t>(), h->d_g_cell0.as<int32_t>(), h->d_cell_start.as<int32_t>(), ev,    \
                     h->d_slot_base.as<int64_t>(), h->d_nl_off.as<int64_t>(), h->d_nl_e.as<int32_t>(),            \
                     h->d_nl_d.as<int32_t>(), h->d_nl_r.as<int32_t>(), jpart, own, gpart, gnp, ng, padded, tab,     \
                     rot, evd, h->d_perm.as<int32_t>(), cap, pairs_out, pcount, mol_count, ws.epoch)
#define AICA_LAUNCH(MIX, COMP) AICA_LAUNCH_R(MIX, COMP, false)
  if (rot) {  // rotating referral: compensated sums always (the variants with a rotation are built once)
    if (nsp == 1) AICA_LAUNCH_R(0, true, true);
    else if (nsp == 2) AICA_LAUNCH_R(1, true, true);
    else AICA_LAUNCH_R(2, true, true);
  } else if (MODE == 1 || comp) {
    if (nsp == 1) AICA_LAUNCH(0, true);
    else if (nsp == 2) AICA_LAUNCH(1, true);
    else AICA_LAUNCH(2, true);
  } else {
    if (nsp == 1) AICA_LAUNCH(0, false);
    else if (nsp == 2) AICA_LAUNCH(1, false);
    else AICA_LAUNCH(2, false);
  }
#undef AICA_LAUNCH
#undef AICA_LAUNCH_R
  HIPCHK(hipGetLastError());
  return AICA_OK;
}

// The adjoint pair kernel (one, two, or three to eight species).
template <typename T>
static int launch_adj(aica_dil *h, const LJTab &tab, const AdjTab &at, hipStream_t st) {
  using V4 = typename Vec4<T>::type;
  const int64_t ng = h->grp.ng;
  constexpr int NW = adj_waves(sizeof(T));
  const int64_t nblocks = (ng + NW - 1) / NW;
  const int64_t padded = ((nblocks + 7) / 8) * 8;
  const V4 *ev = sizeof(T) == 4 ? (const V4 *)h->d_e_vec32.p : (const V4 *)h->d_e_vec64.p;
  const double *rot = h->geo.has_rot ? h->d_rot64.as<double>() : nullptr;
  const double4 *evd = h->geo.has_rot ? h->d_e_vec64.as<double4>() : nullptr;
#define AICA_LAUNCH_ADJ(MIX, ROT)                                                                                   \
  hipLaunchKernelGGL((k_pair_adj<T, MIX, ROT>), dim3((unsigned)padded), dim3(64 * NW), 0, st, h->d_pos.as<V4>(),   \
                     h->d_gG.as<V4>(), h->d_g_start.as<int32_t>(), h->d_g_cell0.as<int32_t>(),                     \
                     h->d_cell_start.as<int32_t>(), ev, h->d_slot_base.as<int64_t>(), h->d_nl_off.as<int64_t>(),    \
                     h->d_nl_e.as<int32_t>(), h->d_nl_d.as<int32_t>(), h->d_nl_r.as<int32_t>(), h->d_jpart.as<double>(), \
                     h->d_own.as<T>(), h->d_gpar.as<double>(), ng, padded, tab, at, rot, evd, h->epoch)
  if (rot) {
    if (tab.nsp == 1) AICA_LAUNCH_ADJ(0, true);
    else if (tab.nsp == 2) AICA_LAUNCH_ADJ(1, true);
    else AICA_LAUNCH_ADJ(2, true);
  } else {
    if (tab.nsp == 1) AICA_LAUNCH_ADJ(0, false);
    else if (tab.nsp == 2) AICA_LAUNCH_ADJ(1, false);
    else AICA_LAUNCH_ADJ(2, false);
  }
#undef AICA_LAUNCH_ADJ
  HIPCHK(hipGetLastError());
  return AICA_OK;
}

template <typename T, bool COMP>
static void launch_finalize(aica_dil *h, const ForceWs &ws, void *out, hipStream_t st) {
  const int64_t n = h->n;
  hipLaunchKernelGGL((k_finalize<T, COMP>), dim3(grid1d(n, 256)), dim3(256), 0, st, (const T *)ws.own,
                     (const T *)ws.jpart, h->jtotal, n, h->d_cell_sorted.as<int32_t>(), h->d_cell_start.as<int32_t>(),
                     h->d_slot_base.as<int64_t>(), h->d_rcnt.as<int32_t>(), h->d_perm.as<int32_t>(), (T *)out,
                     ws.epoch);
}

// Gather the binned positions into cell-sorted SoA at dst ([n] V4 of the compute type).
template <typename T>
static int gather_to(aica_dil *h, const void *pos_dev, const int32_t *species, int tab_nsp, hipStream_t st, void *dst) {
  using V4 = typename Vec4<T>::type;
  const int64_t n = h->n;
  if (n == 0) return AICA_OK;
  if (h->bin_dtype == AICA_FP64)
    hipLaunchKernelGGL((k_gather<T, double>), dim3(grid1d(n, 256)), dim3(256), 0, st, (const double *)pos_dev, species,
                       h->d_perm.as<int32_t>(), h->d_mol_group.as<int32_t>(), h->d_orig.as<double>(), n, tab_nsp, (V4 *)dst);
  else
    hipLaunchKernelGGL((k_gather<T, float>), dim3(grid1d(n, 256)), dim3(256), 0, st, (const float *)pos_dev, species,
                       h->d_perm.as<int32_t>(), h->d_mol_group.as<int32_t>(), h->d_orig.as<double>(), n, tab_nsp, (V4 *)dst);
  HIPCHK(hipGetLastError());
  return AICA_OK;
}

// Gather into the handle's own position buffer (grown as needed).
template <typename T>
static int gather(aica_dil *h, const void *pos_dev, const int32_t *species, int tab_nsp, hipStream_t st) {
  using V4 = typename Vec4<T>::type;
  int rc = h->d_pos.ensure(sizeof(V4) * std::max<int64_t>(h->n, 1));
  if (rc) return rc;
  return gather_to<T>(h, pos_dev, species, tab_nsp, st, h->d_pos.p);
}

// The handle's grow-only workspace for a force call (allocating on first use or growth).
template <typename T>
static int handle_ws(aica_dil *h, ForceWs &ws, hipStream_t st) {
  const int64_t n = h->n, ng = h->grp.ng, J = h->jtotal;
  int rc;
  if ((rc = prepare_jpart(h, sizeof(T) * 4 * std::max<int64_t>(J, 1), st))) return rc;
  if ((rc = h->d_own.ensure(sizeof(T) * 8 * std::max<int64_t>(n, 1)))) return rc;
  if ((rc = h->d_gpart.ensure(sizeof(double) * 2 * std::max<int64_t>(ng, 1)))) return rc;
  if ((rc = h->d_gnp.ensure(16 * std::max<int64_t>(ng, 1)))) return rc;
  if ((rc = h->d_red.ensure(sizeof(double) * 8 * kRedBlocks))) return rc;
  ws.pos = h->d_pos.p;
  ws.own = h->d_own.p;
  ws.jpart = h->d_jpart.p;
  ws.gpart = h->d_gpart.p;
  ws.gnp = h->d_gnp.p;
  ws.red = h->d_red.p;
  ws.epoch = h->epoch;
  return AICA_OK;
}

static int check_step(aica_dil *h, const void *pos_dev) {
  if (!h) return fail(AICA_E_INVAL, "handle is NULL");
  if (!h->bin_valid) return fail(AICA_E_INVAL, "aica_bin must succeed before this call");
  if (pos_dev != h->bin_pos) return fail(AICA_E_INVAL, "positions differ from the array passed to aica_bin");
  return AICA_OK;
}

// Pair kernel, finalize and reductions of a force call on the workspace ws (positions already gathered).
template <typename T>
static int forces_impl(aica_dil *h, const ForceWs &ws, const LJTab &tab, bool comp, void *forces_dev, double *uw_dev,
                       int64_t *npairs_dev, hipStream_t st, bool prof = true) {
  const int64_t n = h->n, ng = h->grp.ng;
  int rc;
  const bool was = h->profiling;
  h->profiling = was && prof;  // the timing events are created only where the call may allocate
  struct Restore {
    aica_dil *h;
    bool v;
    ~Restore() { h->profiling = v; }
  } restore{h, was};
  {
    ProfScope ps(h, "pair_fwd", st);
    if ((rc = launch_pair<T, 0>(h, ws, tab, comp, st, 0, nullptr))) return rc;
    h->wsteps_valid = ws.gnp == h->d_gnp.p;  // the lane-pair diagnostic reads the handle's partials
  }
  {
    ProfScope ps(h, "finalize", st);
    if (n > 0 && forces_dev) {
      if (comp && sizeof(T) == 4)
        launch_finalize<T, true>(h, ws, forces_dev, st);
      else
        launch_finalize<T, false>(h, ws, forces_dev, st);
    }
    if (uw_dev || npairs_dev) {
      int64_t chunk;
      const int nb = red_blocks(ng, chunk);
      double *pu = (double *)ws.red, *pn = pu + 2 * kRedBlocks;
      hipLaunchKernelGGL((k_reduce_rows<2, double>), dim3(nb), dim3(kRedThreads), 0, st, (const double *)ws.gpart, ng,
                         2, 0, chunk, pu);
      hipLaunchKernelGGL((k_reduce_rows<1, unsigned long long>), dim3(nb), dim3(kRedThreads), 0, st,
                         (const unsigned long long *)ws.gnp, ng, 2, 0, chunk, pn);
      hipLaunchKernelGGL(k_reduce_uw, dim3(1), dim3(kRedThreads), 0, st, pu, pn, nb, uw_dev, npairs_dev);
    }
    HIPCHK(hipGetLastError());
  }
  return AICA_OK;
}

template <typename T>
static int forces_alloc(aica_dil *h, const void *pos_dev, const int32_t *species, const LJTab &tab, bool comp,
                        void *forces_dev, double *uw_dev, int64_t *npairs_dev, hipStream_t st) {
  int rc;
  if ((rc = gather<T>(h, pos_dev, species, tab.nsp, st))) return rc;
  ForceWs ws;
  if ((rc = handle_ws<T>(h, ws, st))) return rc;
  return forces_impl<T>(h, ws, tab, comp, forces_dev, uw_dev, npairs_dev, st);
}

int aica_forces(aica_dil *h, const void *pos_dev, const int32_t *species_dev, const aica_params *params,
                void *forces_dev, double *uw_dev, int64_t *npairs_dev, void *hip_stream) {
  int rc = check_step(h, pos_dev);
  if (rc) return rc;
  LJTab tab;
  if ((rc = build_tab(h, params, tab))) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  if (params->precision == AICA_FP32)
    return forces_alloc<float>(h, pos_dev, species_dev, tab, params->compensated != 0, forces_dev, uw_dev, npairs_dev, st);
  return forces_alloc<double>(h, pos_dev, species_dev, tab, false, forces_dev, uw_dev, npairs_dev, st);
}

// ---- aica_forces without allocation: every buffer of the call lies in this fixed array (one copy per GPU,
// held until the process ends).  Host code never passes the array's name to a kernel: it resolves the
// array's device address once per device (hipGetSymbolAddress) and uses that.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static void *g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

static int scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(AICA_E_INVAL, "device index out of range for the scratch array");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(AICA_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return AICA_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

template <typename T>
static int forces_noalloc(aica_dil *h, const void *pos_dev, const int32_t *species, const LJTab &tab, bool comp,
                          void *forces_dev, double *uw_dev, int64_t *npairs_dev, hipStream_t st) {
  using V4 = typename Vec4<T>::type;
  const int64_t n = h->n, ng = h->grp.ng, J = h->jtotal;
  const size_t b_pos = align256(sizeof(V4) * std::max<int64_t>(n, 1));
  const size_t b_own = align256(sizeof(T) * 8 * std::max<int64_t>(n, 1));
  const size_t b_jpart = align256(sizeof(T) * 4 * std::max<int64_t>(J, 1));
  const size_t b_gpart = align256(sizeof(double) * 2 * std::max<int64_t>(ng, 1));
  const size_t b_gnp = align256(16 * std::max<int64_t>(ng, 1));
  const size_t b_red = align256(sizeof(double) * 8 * kRedBlocks);
  const size_t need = b_pos + b_own + b_jpart + b_gpart + b_gnp + b_red;
  if (need > kScratchBytes)
    return fail(AICA_E_INVAL, "aica_forces_noalloc needs " + std::to_string(need) + " bytes of scratch for " +
                                  std::to_string(n) + " molecules; the fixed scratch holds " +
                                  std::to_string(kScratchBytes) + " (use aica_forces)");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  char *base = nullptr;
  int rc = scratch_address(dev, (void **)&base);
  if (rc) return rc;
  ForceWs ws;
  ws.pos = base;
  ws.own = base + b_pos;
  ws.jpart = base + b_pos + b_own;
  ws.gpart = base + b_pos + b_own + b_jpart;
  ws.gnp = base + b_pos + b_own + b_jpart + b_gpart;
  ws.red = base + b_pos + b_own + b_jpart + b_gpart + b_gnp;
  // the array keeps the last call's records: every record's tag is cleared (a fill kernel, no memset node)
  ws.epoch = 1;
  const int64_t words = (int64_t)(sizeof(T) * 4 * std::max<int64_t>(J, 1) / 4);
  hipLaunchKernelGGL((k_fill<uint32_t>), dim3(grid1d(words, 256)), dim3(256), 0, st, (uint32_t *)ws.jpart, words,
                     0xFFFFFFFFu);
  HIPCHK(hipGetLastError());
  if ((rc = gather_to<T>(h, pos_dev, species, tab.nsp, st, ws.pos))) return rc;
  return forces_impl<T>(h, ws, tab, comp, forces_dev, uw_dev, npairs_dev, st, false);
}

int aica_forces_noalloc(aica_dil *h, const void *pos_dev, const int32_t *species_dev, const aica_params *params,
                        void *forces_dev, double *uw_dev, int64_t *npairs_dev, void *hip_stream) {
  int rc = check_step(h, pos_dev);
  if (rc) return rc;
  LJTab tab;
  if ((rc = build_tab(h, params, tab))) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  if (params->precision == AICA_FP32)
    return forces_noalloc<float>(h, pos_dev, species_dev, tab, params->compensated != 0, forces_dev, uw_dev, npairs_dev, st);
  return forces_noalloc<double>(h, pos_dev, species_dev, tab, false, forces_dev, uw_dev, npairs_dev, st);
}

int aica_pairs_export(aica_dil *h, const void *pos_dev, const aica_params *params, int64_t cap, int64_t *n_out,
                      int32_t *a, int32_t *b, int8_t *img, void *hip_stream) {
  int rc = check_step(h, pos_dev);
  if (rc) return rc;
  if (!n_out || cap < 0 || (cap > 0 && (!a || !b || !img))) return fail(AICA_E_INVAL, "bad output arrays");
  LJTab tab;
  if ((rc = build_tab(h, params, tab))) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  if ((rc = h->d_pairs.ensure(12 * std::max<int64_t>(cap, 1)))) return rc;
  if ((rc = h->d_pcount.ensure(64))) return rc;
  unsigned long long *pc = h->d_pcount.as<unsigned long long>();
  hipLaunchKernelGGL((k_fill<unsigned long long>), dim3(1), dim3(64), 0, st, pc, (int64_t)1, 0ull);
  if (params->precision == AICA_FP32) {
    if ((rc = gather<float>(h, pos_dev, nullptr, 1, st))) return rc;
    ForceWs ws;
    ws.pos = h->d_pos.p;
    if ((rc = launch_pair<float, 1>(h, ws, tab, false, st, cap, pc))) return rc;
  } else {
    if ((rc = gather<double>(h, pos_dev, nullptr, 1, st))) return rc;
    ForceWs ws;
    ws.pos = h->d_pos.p;
    if ((rc = launch_pair<double, 1>(h, ws, tab, false, st, cap, pc))) return rc;
  }
  unsigned long long cnt = 0;
  HIPCHK(hipMemcpyAsync(&cnt, pc, 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  *n_out = (int64_t)cnt;
  const int64_t k = std::min<int64_t>((int64_t)cnt, cap);
  if (k > 0) {
    std::vector<int32_t> buf(3 * k);
    HIPCHK(hipMemcpy(buf.data(), h->d_pairs.p, 12 * k, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < k; ++i) {
      int32_t x = buf[3 * i], y = buf[3 * i + 1], code = buf[3 * i + 2];
      int n0 = code / 9 - 1, n1 = (code / 3) % 3 - 1, n2 = code % 3 - 1;
      // d = x_i - x_j - t with t = image of the entry; report (min id, max id, image of that order)
      if (x > y) {
        std::swap(x, y);
        n0 = -n0;
        n1 = -n1;
        n2 = -n2;
      }
      a[i] = x;
      b[i] = y;
      img[3 * i] = (int8_t)n0;
      img[3 * i + 1] = (int8_t)n1;
      img[3 * i + 2] = (int8_t)n2;
    }
  }
  return AICA_OK;
}

int aica_forces_adjoint(aica_dil *h, const void *pos_dev, const int32_t *species_dev, const aica_params *params,
                        const void *grad_forces_dev, double grad_energy, void *grad_pos_dev, double *grad_eps_dev,
                        double *grad_sigma_dev, void *hip_stream);

int aica_pair_counts(aica_dil *h, const void *pos_dev, const aica_params *params, int32_t *counts_dev,
                     void *hip_stream) {
  int rc = check_step(h, pos_dev);
  if (rc) return rc;
  if (h->n > 0 && !counts_dev) return fail(AICA_E_INVAL, "counts_dev is NULL");
  LJTab tab;
  if ((rc = build_tab(h, params, tab))) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  if (h->n == 0) return AICA_OK;
  hipLaunchKernelGGL((k_fill<int32_t>), dim3(grid1d(h->n, 256)), dim3(256), 0, st, counts_dev, h->n, 0);
  if (params->precision == AICA_FP32) {
    if ((rc = gather<float>(h, pos_dev, nullptr, 1, st))) return rc;
    ForceWs ws;
    ws.pos = h->d_pos.p;
    if ((rc = launch_pair<float, 1>(h, ws, tab, false, st, -1, nullptr, counts_dev))) return rc;
  } else {
    if ((rc = gather<double>(h, pos_dev, nullptr, 1, st))) return rc;
    ForceWs ws;
    ws.pos = h->d_pos.p;
    if ((rc = launch_pair<double, 1>(h, ws, tab, false, st, -1, nullptr, counts_dev))) return rc;
  }
  HIPCHK(hipGetLastError());
  return AICA_OK;
}

int aica_dil_export(const aica_dil *h, int64_t *n, int32_t *c, int32_t *d, int8_t *img) {
  if (!h || !n) return fail(AICA_E_INVAL, "NULL argument");
  *n = (int64_t)h->pairs.size();
  if (!c) return AICA_OK;
  if (!d || !img) return fail(AICA_E_INVAL, "NULL output array");
  for (size_t i = 0; i < h->pairs.size(); ++i) {
    const CellPair &p = h->pairs[i];
    int32_t x = h->order[p.sc], y = h->order[p.sd];
    int n0 = p.img[0], n1 = p.img[1], n2 = p.img[2];
    if (x > y) {
      std::swap(x, y);
      n0 = -n0;
      n1 = -n1;
      n2 = -n2;
    }
    c[i] = x;
    d[i] = y;
    img[3 * i] = (int8_t)n0;
    img[3 * i + 1] = (int8_t)n1;
    img[3 * i + 2] = (int8_t)n2;
  }
  return AICA_OK;
}

int aica_bin_export(const aica_dil *h, int32_t *cell_of, int32_t *order, int64_t *cell_count) {
  if (!h) return fail(AICA_E_INVAL, "handle is NULL");
  if (!h->bin_valid) return fail(AICA_E_INVAL, "aica_bin must succeed first");
  const int64_t n = h->n, nc = h->geo.nc;
  if (cell_of && n > 0) {
    std::vector<int32_t> cs(n), pm(n);
    HIPCHK(hipMemcpy(cs.data(), h->d_cell_sorted.p, 4 * n, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(pm.data(), h->d_perm.p, 4 * n, hipMemcpyDeviceToHost));
    for (int64_t s = 0; s < n; ++s) cell_of[pm[s]] = h->order[cs[s]];
  }
  if (order && n > 0) HIPCHK(hipMemcpy(order, h->d_perm.p, 4 * n, hipMemcpyDeviceToHost));
  if (cell_count) {
    std::vector<int32_t> cs(nc + 1);
    HIPCHK(hipMemcpy(cs.data(), h->d_cell_start.p, 4 * (nc + 1), hipMemcpyDeviceToHost));
    for (int64_t s = 0; s < nc; ++s) cell_count[h->order[s]] = cs[s + 1] - cs[s];
  }
  return AICA_OK;
}

int aica_dil_info(const aica_dil *h, aica_info *info) {
  if (!h || !info) return fail(AICA_E_INVAL, "NULL argument");
  memset(info, 0, sizeof *info);
  info->n_cells = h->geo.nc;
  info->n_dil = (int64_t)h->pairs.size();
  info->n_groups = h->groups_ready ? h->grp.ng : 0;
  info->n_group_pairs = h->groups_ready ? h->grp.e_off[h->grp.ng] : 0;
  info->n_molecules = h->n;
  info->n_jslots = h->jtotal;
  info->mesh_volume = h->geo.total_volume;
  info->build_seconds = h->build_seconds;
  info->group_seconds = h->group_seconds;
  info->lane_steps = -1;
  info->located_ball = h->located[0];
  info->located_record = h->located[1];
  info->located_search = h->located[2];
  return AICA_OK;
}

int aica_work_stats(const aica_dil *h, int64_t *dil_candidates, int64_t *lane_pairs) {
  if (!h) return fail(AICA_E_INVAL, "handle is NULL");
  if (!h->bin_valid) return fail(AICA_E_INVAL, "aica_bin must succeed first");
  const int64_t nc = h->geo.nc, ng = h->grp.ng;
  std::vector<int32_t> cs(nc + 1), gs(ng + 1);
  HIPCHK(hipMemcpy(cs.data(), h->d_cell_start.p, 4 * (nc + 1), hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(gs.data(), h->d_g_start.p, 4 * (ng + 1), hipMemcpyDeviceToHost));
  if (dil_candidates) {
    int64_t cand = 0;
    for (int64_t s = 0; s < nc; ++s) {
      const int64_t n = cs[s + 1] - cs[s];
      cand += n * (n - 1) / 2;
    }
    for (const CellPair &p : h->pairs) cand += (int64_t)(cs[p.sc + 1] - cs[p.sc]) * (cs[p.sd + 1] - cs[p.sd]);
    *dil_candidates = cand;
  }
  if (lane_pairs) {
    // wave-steps counted by the last forward pair kernel, 64 lane-pair evaluations each
    if (!h->wsteps_valid) return fail(AICA_E_INVAL, "aica_forces must run after aica_bin first");
    std::vector<unsigned long long> gn(2 * ng);
    HIPCHK(hipMemcpy(gn.data(), h->d_gnp.p, 16 * ng, hipMemcpyDeviceToHost));
    int64_t lp = 0;
    for (int64_t a = 0; a < ng; ++a) lp += 64 * (int64_t)gn[2 * a + 1];
    *lane_pairs = lp;
  }
  return AICA_OK;
}

int aica_profile(aica_dil *h, int32_t enable) {
  if (!h) return fail(AICA_E_INVAL, "handle is NULL");
  h->profiling = enable != 0;
  return AICA_OK;
}

int aica_profile_read(aica_dil *h, const char *kernel, double *ms_total, int64_t *launches, int32_t reset) {
  if (!h || !kernel) return fail(AICA_E_INVAL, "NULL argument");
  Timer &t = h->timers[kernel];
  for (auto &ev : t.pending) {
    HIPCHK(hipEventSynchronize(ev.second));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, ev.first, ev.second));
    t.ms += ms;
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  t.pending.clear();
  if (ms_total) *ms_total = t.ms;
  if (launches) *launches = t.launches;
  if (reset) {
    t.ms = 0;
    t.launches = 0;
  }
  return AICA_OK;
}


#include "aica_adjoint.inc"
