/*
 * aica.h - C ABI of the MI355X-native AICA Lennard-Jones pair-force library.
 *
 * The Arbitrary Interacting Cells Algorithm (Macpherson & Reese, arXiv
 * cs/0702131) evaluates short-range pair forces for molecules held in the
 * cells of a static, unstructured, arbitrary polyhedral mesh (Sec. 2.2, 2.3).
 * Each cell interacts with itself and with the cells on its direct
 * interaction list (DIL), every cell pair being listed once (Sec. 2.2,
 * App. A.1); periodic boundaries are handled by referred cells, i.e. images
 * of real cells under the boundary's referring transform (Sec. 2.1, 2.2.1,
 * 2.2.2).  On one GPU only periodic referral exists; each periodic direction
 * has one transform in the generic form P' = y + R.P of Sec. 2.2.2: a lattice
 * translation (R = I) or a rotation about an axis (coupled boundaries that
 * are not parallel, e.g. the two sides of a sector of a rotationally
 * symmetric domain).
 *
 * Conventions for every call:
 *   - Return value: AICA_OK (0) or a negative AICA_E_* code; nothing throws.
 *     aica_last_error() gives a message for the calling thread.
 *   - "host" pointers are CPU memory; "device" pointers are HIP device memory
 *     (e.g. torch tensor data pointers).  The caller owns all arrays; the
 *     library owns the aica_dil handle and everything inside it.
 *   - Device work is stream-ordered on the caller's HIP stream (hipStream_t
 *     passed as void*; NULL means the legacy default stream).
 *   - Molecule ids are 0..n-1 in the caller's order; results come back in the
 *     caller's order.  Cell ids are the mesh's own cell indices.
 */
#ifndef AICA_H
#define AICA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AICA_OK 0
#define AICA_E_INVAL -1      /* bad argument: null pointer, size, dtype, NaN position, wrong call order */
#define AICA_E_MESH -2       /* invalid mesh: bad indices, open or inverted cell (non-positive tetrahedron) */
#define AICA_E_RCUT -3       /* rcut + guard >= half a periodic length (minimum image would not hold) */
#define AICA_E_UNLOCATED -4  /* some molecule lies in no cell of the mesh */
#define AICA_E_NOMEM -5      /* host or device allocation failed */
#define AICA_E_HIP -6        /* a HIP runtime call failed */

#define AICA_FP32 1
#define AICA_FP64 2

/* Static unstructured polyhedral mesh (Sec. 2.3: a cell's index implies
 * nothing about its location or connectivity).  Host memory, read during
 * aica_build_dil only and not retained. */
typedef struct aica_mesh {
  int64_t n_points;
  const double *points;      /* [n_points][3] */
  int64_t n_faces;
  const int64_t *face_off;   /* [n_faces+1]: face f uses face_pts[face_off[f] .. face_off[f+1]) */
  const int32_t *face_pts;   /* vertex loops; right-hand normal points out of the owner cell */
  const int32_t *owner;      /* [n_faces] owning cell */
  const int32_t *neighbour;  /* [n_faces] other cell, or -1 on a boundary face */
  int64_t n_cells;
  int32_t n_periodic;        /* number of periodic directions (0..3) */
  double periodic_vec[3][3]; /* y_k: the shift of direction k's referring transform x -> R_k x + y_k */
  const double *periodic_rot;/* NULL (every R_k = I: lattice translations, which must be mutually
                                orthogonal), or [n_periodic][3][3] row-major R_k.  A rotation (R_k != I)
                                must be proper (orthonormal, det +1) and of finite order K_k <= 64 with
                                K_k >= 3 (T_k^K = identity; T_k and its inverse distinct), and the
                                transforms of all directions must commute.  Image n of a cell is
                                T_1^n_1 T_2^n_2 T_3^n_3 with n_k in {-1, 0, 1}. */
} aica_mesh;

/* Lennard-Jones model and evaluation options.  Host memory. */
typedef struct aica_params {
  double rcut;               /* cut-off radius, absolute, the same for every species pair; <= the DIL's rcut */
  int32_t n_species;         /* 1..8 */
  const double *eps;         /* [n_species] per-species epsilon (Lorentz-Berthelot: eps_ab = sqrt(eps_a eps_b)) */
  const double *sigma;       /* [n_species] per-species sigma (sigma_ab = (sigma_a + sigma_b)/2) */
  int32_t precision;         /* AICA_FP32: FP32 pair arithmetic, compensated FP32 force sums, FP64 energy and
                                virial; AICA_FP64: FP64 throughout */
  int32_t compensated;       /* FP32 only: 1 = TwoSum-compensated per-molecule force sums, 0 = plain FP32 */
} aica_params;

typedef struct aica_dil aica_dil;  /* opaque handle */

/* Setup (Sec. 2.3 and App. A): validate the mesh, build every cell's direct
 * interaction list and the periodic referred-cell pairs, once.  A cell pair
 * (c, d, n), n the image powers with components in {-1,0,1}, is listed when
 * the closest distance between cell c and cell d mapped by image n is below
 * rcut + guard; each pair is listed once (App. A.1: (c, d, n) and (d, c, -n)
 * are the same pair), and no cell is listed with itself at n = 0.  Images
 * beyond the first powers must be out of range: for lattice translations
 * rcut + guard must be below half of every periodic length, and with a
 * rotation no cell pair may be in range through any other power of the
 * transforms (checked; AICA_E_RCUT otherwise).  Cell geometry: each face is fanned into
 * triangles around the mean of its vertices; the cell is the union of the
 * tetrahedra (cell vertex mean, face triangle), all of which must have
 * positive volume.  rcut > 0 is the largest cut-off of any potential
 * (App. A); guard >= 0 widens the list (Sec. 2.2 guard distance).
 * Errors: AICA_E_INVAL, AICA_E_MESH, AICA_E_RCUT, AICA_E_NOMEM, AICA_E_HIP.
 * On success *out owns device geometry and must be freed with aica_dil_free. */
int aica_build_dil(const aica_mesh *mesh, double rcut, double guard, aica_dil **out);

#define AICA_DIL_CLOSEST 0  /* closest distance between the closed cells (no pair can be missed) */
#define AICA_DIL_VERTEX 1   /* the paper's own test: some vertex of c and some vertex of d + t closer */

/* aica_build_dil with a choice of cell-pair predicate.  AICA_DIL_VERTEX is the
 * test of Sec. 2.2 and App. A.1 (vertex-to-vertex distance below rcut + guard);
 * on distorted meshes it can miss cell pairs whose closest points are within
 * range while all their vertices are not (Sec. 2.2 on twisted meshes), and
 * then molecule pairs inside the cut-off go unevaluated.  Everything else as
 * aica_build_dil (which is predicate AICA_DIL_CLOSEST).
 * Errors: as aica_build_dil, plus AICA_E_INVAL for an unknown predicate. */
int aica_build_dil_ex(const aica_mesh *mesh, double rcut, double guard, int32_t predicate, aica_dil **out);

/* Per-step binning (Sec. 2.2: the library keeps which cell each molecule is
 * in).  pos_dev: device [n][3] positions in the caller's order, dtype
 * AICA_FP64 (double) or AICA_FP32 (float); every position must lie in the
 * mesh (periodic coordinates already wrapped by the caller).  Locates each
 * molecule's cell (lowest cell index on a shared face), builds the CSR cell
 * occupancy and the cell-sorted order (ascending molecule id within a cell),
 * and the per-step work list.  Results stay in the handle.  Membership is
 * tracked from the previous call with the same n (Sec. 2.2): a molecule still
 * inside the ball kept from its last record test in its previous cell needs
 * no test at all; otherwise the previous cell is tested first, then the cells
 * across its faces, then a background grid.  The answer does not depend on
 * the history (every route certifies the same cell).  A cell may hold any
 * number of molecules.  Synchronises the stream once, to read the unlocated
 * and reaction-slot counts.
 * Errors: AICA_E_INVAL (n < 0 or n >= 2^28 - 1, null, bad dtype),
 * AICA_E_UNLOCATED (the count is in aica_last_error), AICA_E_NOMEM (more than
 * 2^31 reaction records), AICA_E_HIP. */
int aica_bin(aica_dil *dil, const void *pos_dev, int32_t pos_dtype, int64_t n, void *hip_stream);

/* Per-step forces (Sec. 2.3.1 real-real and 2.3.2 real-referred loops, with
 * the reaction -F applied to the partner, Sec. 2.2): for every unordered pair
 * {a, T b} (T the image's referring transform x -> R x + y) with
 * |d|^2 < rcut^2, d = x_a - T x_b,
 *   u = 4 eps_ab [(sigma_ab/r)^12 - (sigma_ab/r)^6],  F_a += g d, F_b -= R^T g d,
 *   g = 24 eps_ab [2 sigma_ab^12 r^-14 - sigma_ab^6 r^-8],
 *   U = sum u, W = sum g |d|^2 (virial sum r.F), npairs = number of pairs.
 * pos_dev must be the array last passed to aica_bin (same pointer, dtype and
 * n; otherwise AICA_E_INVAL).  species_dev: device int32 [n] in 0..n_species-1,
 * or NULL for all-zero; the ids are not checked (that would cost a synchronisation):
 * an id below 0 is taken as 0 and one above n_species-1 as n_species-1.  forces_dev: device [n][3] in the compute precision's
 * dtype (float for AICA_FP32, double for AICA_FP64), caller order, overwritten.
 * uw_dev: device double[2] = {U, W}, overwritten; npairs_dev: device int64,
 * overwritten.  Either may be NULL.  Results are deterministic (fixed
 * summation order, no atomics on forces).  With AICA_FP32 the cut-off is still
 * decided exactly for positions that are multiples of 2^-15 (pairs within
 * 2^-20 rc^2 of rc^2 are decided in FP64), except for images with a rotation:
 * a rotated position is formed in FP64 and kept as an FP32 value plus its FP32
 * remainder (the adjoint forms the pair vector from both), so only a pair
 * within about 1e-7 rc^2 of rc^2 may be decided either way.
 * Errors: AICA_E_INVAL, AICA_E_NOMEM, AICA_E_HIP. */
int aica_forces(aica_dil *dil, const void *pos_dev, const int32_t *species_dev, const aica_params *params,
                void *forces_dev, double *uw_dev, int64_t *npairs_dev, void *hip_stream);

/* aica_forces for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): same
 * arguments, preconditions and results (bit for bit) as aica_forces, but every
 * buffer of the call lies in a fixed device array of 128 MiB that the library
 * holds on each GPU it runs on until the process ends; the call allocates and
 * frees nothing.  The array holds the cell-sorted positions (16 or 32 bytes per
 * molecule), the own records (32 or 64 bytes per molecule), the reaction records
 * (16 or 32 bytes each, aica_info.n_jslots of them) and per-group partials
 * (32 bytes per group), each region rounded up to 256 bytes, plus 32 KiB; a step
 * that needs more fails with AICA_E_INVAL (the message names the bytes needed)
 * and nothing is launched.  The handle and its binning (aica_build_dil, aica_bin)
 * are prepared beforehand by those calls, which may allocate.  The array keeps
 * the last call's contents; each call first clears the reaction records' tags
 * (a fill kernel, no memset).  All calls on one GPU share the array: calls that
 * overlap in time on one GPU (other streams, other threads, other handles) race
 * and give wrong results; order them on one stream.  aica_profile timing is not
 * recorded for this call.  Errors: AICA_E_INVAL, AICA_E_HIP. */
int aica_forces_noalloc(aica_dil *dil, const void *pos_dev, const int32_t *species_dev, const aica_params *params,
                        void *forces_dev, double *uw_dev, int64_t *npairs_dev, void *hip_stream);

/* Adjoint of the force evaluation for L = sum_a G_a . F_a + gamma U (the
 * upstream gradient G on the forces and gamma on the energy).  Recomputes
 * every pair term (nothing is stored between the calls):
 *   dL/dx_a, dL/deps_s, dL/dsigma_s (per species, through Lorentz-Berthelot).
 * grad_forces_dev: device [n][3] in the compute dtype (G), caller order.
 * grad_energy: gamma (host scalar).  grad_pos_dev: device [n][3] compute dtype,
 * overwritten.  grad_eps_dev, grad_sigma_dev: device double[n_species],
 * overwritten (either may be NULL).  Same preconditions as aica_forces
 * (1..8 species).  Precision: the pair terms (which carry up
 * to r^-16) are formed in FP64 in both precisions, from the FP32 positions and G
 * with AICA_FP32 (whose differences are exact for multiples of 2^-15), and summed
 * per molecule in FP64; with AICA_FP32 only the roundings of the per-entry
 * partial sums and of the result to FP32 remain.  The parameter gradients are
 * the per species-pair sums of dl/deps_ab and dl/dsigma_ab (FP64) taken back to
 * the species through the mixing rule (d eps_ab/d eps_a = eps_ab/(2 eps_a) and
 * d sigma_ab/d sigma_a = 1/2 for a != b).
 * Errors: AICA_E_INVAL, AICA_E_NOMEM, AICA_E_HIP. */
int aica_forces_adjoint(aica_dil *dil, const void *pos_dev, const int32_t *species_dev, const aica_params *params,
                        const void *grad_forces_dev, double grad_energy, void *grad_pos_dev, double *grad_eps_dev,
                        double *grad_sigma_dev, void *hip_stream);

/* ---- diagnostics (tests and benchmarks) ---- */

/* The interacting cell pairs in mesh cell ids: (c, d, img) with c < d, or
 * c == d and img lexicographically positive; img[3] holds the powers of the
 * periodic directions' transforms.  Host arrays.  With c == NULL only *n is set. */
int aica_dil_export(const aica_dil *dil, int64_t *n, int32_t *c, int32_t *d, int8_t *img);

/* The molecule pairs the GPU path evaluates inside the cut-off, as (a, b, img)
 * with d = x_a - T_img x_b (a and b in either order; a == b for a molecule and
 * its own image).  Runs the same traversal as
 * aica_forces after aica_bin.  Host output arrays of capacity cap; *n gets the
 * count (which may exceed cap: call again with a larger cap). */
int aica_pairs_export(aica_dil *dil, const void *pos_dev, const aica_params *params, int64_t cap, int64_t *n,
                      int32_t *a, int32_t *b, int8_t *img, void *hip_stream);

/* Per-molecule pair counts: counts_dev[a] = the number of pairs inside the cut-off that molecule a takes
 * part in (each pair counts for both molecules; a molecule paired with its own image counts twice), from
 * the same traversal as aica_forces after aica_bin.  counts_dev: device int32 [n], caller order,
 * overwritten.  params: rcut and precision are used (the cut-off is decided as aica_forces decides it).
 * Same preconditions as aica_forces.  Errors: AICA_E_INVAL, AICA_E_NOMEM, AICA_E_HIP. */
int aica_pair_counts(aica_dil *dil, const void *pos_dev, const aica_params *params, int32_t *counts_dev,
                     void *hip_stream);

/* Binning of the last aica_bin, host arrays: cell_of[n] (mesh cell id of each
 * molecule), order[n] (molecule ids in cell-sorted order), cell_count[n_cells]
 * (molecules per mesh cell).  Any pointer may be NULL. */
int aica_bin_export(const aica_dil *dil, int32_t *cell_of, int32_t *order, int64_t *cell_count);

typedef struct aica_info {
  int64_t n_cells, n_dil, n_groups, n_group_pairs, n_molecules, n_jslots;
  double mesh_volume, build_seconds, group_seconds;
  int64_t lane_steps;       /* reserved (-1) */
  /* how the last aica_bin located its molecules: inside the ball kept from the
   * molecule's last record test in the same cell (no geometry read), by the
   * previous cell's FP32 record, or by the slow path (FP64 record, face
   * neighbours, background grid) */
  int64_t located_ball, located_record, located_search;
} aica_info;
int aica_dil_info(const aica_dil *dil, aica_info *info);

/* Work of the last aica_bin's occupancy, counted on the host:
 *   dil_candidates: molecule pairs the interaction lists make candidates (the method's own
 *                   candidate set: sum over listed cell pairs of n_c n_d, plus n_c (n_c - 1) / 2 per cell);
 *   lane_pairs:     pair evaluations the GPU tiles executed in the last aica_forces on this
 *                   binning (64 per wave-step, padding included; AICA_E_INVAL before one). */
int aica_work_stats(const aica_dil *dil, int64_t *dil_candidates, int64_t *lane_pairs);

/* Kernel timing with HIP events on the caller's stream: enable, then read the
 * accumulated milliseconds and launch count of a named kernel
 * ("pair_fwd", "pair_adj", "bin", "finalize"), and reset. */
int aica_profile(aica_dil *dil, int32_t enable);
int aica_profile_read(aica_dil *dil, const char *kernel, double *ms_total, int64_t *launches, int32_t reset);

const char *aica_last_error(void);
void aica_dil_free(aica_dil *dil);

#ifdef __cplusplus
}
#endif
#endif /* AICA_H */
