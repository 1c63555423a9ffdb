// Internal declarations shared by the host setup code and the HIP launchers.
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <string>
#include <thread>
#include <vector>

#include "aica.h"

namespace aica {

// Thread-local error text; every ABI entry point returns a status code.
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

// Number of host worker threads for setup (AICA_THREADS, else OMP_NUM_THREADS, else hardware).
int host_threads();

// f(begin, end, worker) over [0, n) in dynamically claimed chunks on host_threads() threads.
template <class F>
void parallel_for(int64_t n, F f) {
  const int nt = host_threads();
  if (n < 1024 || nt == 1) {
    f(0, n, 0);
    return;
  }
  std::vector<std::thread> th;
  std::atomic<int64_t> next(0);
  const int64_t chunk = std::max<int64_t>(64, n / (nt * 16));
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t]() {
      for (;;) {
        const int64_t b = next.fetch_add(chunk);
        if (b >= n) break;
        f(b, std::min(n, b + chunk), t);
      }
    });
  for (auto &x : th) x.join();
}

// A referring transform x -> R x + y (the generic form of Sec. 2.2.2); rot == false means R = I.
struct Xf {
  double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  double y[3] = {0, 0, 0};
  bool rot = false;
  void apply(const double *x, double *o) const {
    if (!rot) {
      for (int q = 0; q < 3; ++q) o[q] = x[q] + y[q];
      return;
    }
    double t[3];
    for (int q = 0; q < 3; ++q) t[q] = R[3 * q] * x[0] + R[3 * q + 1] * x[1] + R[3 * q + 2] * x[2] + y[q];
    for (int q = 0; q < 3; ++q) o[q] = t[q];
  }
  Xf inverse() const;                 // x = R^T (x' - y)
  Xf then(const Xf &b) const;         // b after this: x -> b(this(x))
};

// Host copy of the mesh plus derived cell geometry (Sec. 2.3: static mesh).
struct Geometry {
  int64_t np = 0, nf = 0, nc = 0;
  std::vector<double> pts;       // [np][3]
  std::vector<int64_t> foff;     // [nf+1]
  std::vector<int32_t> fpts;     // vertex loops
  std::vector<int32_t> own, nei; // [nf]
  int nper = 0;
  double per[3][3] = {{0}};      // y_k of each periodic direction's transform
  Xf gen[3];                     // the transforms T_k themselves
  int order[3] = {0, 0, 0};      // K_k for a rotation (T_k^K = identity), 0 for a translation
  bool has_rot = false;          // some direction refers with a rotation
  // derived
  std::vector<double> fcen;      // [nf][3] face vertex mean
  std::vector<int64_t> cf_off;   // [nc+1] faces of each cell
  std::vector<int32_t> cf;       // face ids
  std::vector<int8_t> cf_sgn;    // +1: cell owns the face (loop outward), -1: neighbour (loop reversed)
  std::vector<double> ccen;      // [nc][3] vertex mean of the cell's distinct vertices
  std::vector<double> lo, hi;    // [nc][3] bounding boxes
  std::vector<double> vol;       // [nc] cell volumes (sum of tetrahedra)
  std::vector<double> r_in;      // [nc] radius of a ball about the centroid inside the cell
  std::vector<double> r_out;     // [nc] largest centroid-to-vertex distance
  std::vector<int64_t> cv_off;   // [nc+1] distinct vertices of each cell
  std::vector<int32_t> cv;
  double dom_lo[3], dom_hi[3];   // mesh bounding box
  double max_half_ext[3];        // largest cell half extent per axis
  double total_volume = 0;
};

// Validate the mesh and fill the derived geometry.  Returns AICA_OK or an error code.
int build_geometry(const aica_mesh *m, Geometry &g);

// Spatially coherent cell order (k-d median splits of cell centroids):
// order[s] = mesh cell at sorted position s; rank[c] = sorted position of mesh cell c.
void spatial_order(const Geometry &g, std::vector<int32_t> &order, std::vector<int32_t> &rank,
                   std::vector<uint8_t> &split_depth);

// Image n of the periodic directions: T_1^n0 T_2^n1 T_3^n2 (the transforms commute).
Xf image_transform(const Geometry &g, int n0, int n1, int n2);

// One interacting cell pair in sorted cell indices: sc < sd, or sc == sd with img > 0 (lexicographic).
struct CellPair {
  int32_t sc, sd;
  int8_t img[3];
};

// Build the direct interaction lists (App. A.1 with the closest-point predicate and
// guard of Sec. 2.2) including periodic referred pairs (lattice translations).
int build_cell_pairs(const Geometry &g, const std::vector<int32_t> &order, const std::vector<int32_t> &rank,
                     double R, int predicate, std::vector<CellPair> &out);

// Interaction groups: consecutive sorted cells packed to an expected occupancy target.
struct Groups {
  int64_t ng = 0;
  std::vector<int32_t> cell0;   // [ng+1] first sorted cell of each group
  std::vector<int32_t> of_cell; // [nc] group of each sorted cell
  std::vector<double> orig;     // [ng][3] group origin (multiple of 2^-15)
  // group-pair list (CSR by the i-group A)
  std::vector<int64_t> e_off;   // [ng+1]
  std::vector<int32_t> e_B;     // j-group
  std::vector<int8_t> e_img;    // [E][3] lattice multiples
  std::vector<int64_t> r_off;   // [ng+1] reverse list: entries whose j-group is B
  std::vector<int32_t> r_e;     // entry ids
  // needed j-cells: for every non-self entry e = (A, B, t), the cells d of B with some cell of A in
  // range of d + t (CSR by the i-group A, sorted by (e, d))
  std::vector<int64_t> nl_off;  // [ng+1]
  std::vector<int32_t> nl_e;    // entry id
  std::vector<int32_t> nl_d;    // sorted cell id (in group B)
  std::vector<int32_t> nl_r;    // 1 + rank of the entry in the cell's reverse list (0 is the self entry)
  // reverse of the needed lists by cell: entries whose needed list holds cell d
  std::vector<int64_t> rc_off;  // [nc+1]
  std::vector<int32_t> rc_e;
};

int build_groups(const Geometry &g, const std::vector<int32_t> &order, const std::vector<uint8_t> &split_depth,
                 const std::vector<CellPair> &pairs, double density, double target, Groups &out);

}  // namespace aica
