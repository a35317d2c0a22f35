// Device-side data structures and kernel entry points of the sweep library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace vefk {

// Per-problem constant data (device pointers), one entry per problem of a handle.
struct KProb {
  int ne, nd, nbf, n, Q, nq, p, pointwise;  // pointwise: upwind side per face point (general kernels)
  const void *geo_v;       // T [ne][Q][5]: w J, w adj(F) (row major)
  const void *geo_f;       // T [ne][4][nq][2]: w_s n ds
  const void *geo_a;       // T [ne][16]: J, adj(F) (row major), face chords N_0..N_3 (affine meshes)
  const void *emat;        // T [ne][3 n n + 8 (p+1)^2]: element matrices (general elements, p = 3; layout in
                           // emat.hip), or NULL
  const void *cls_inv;     // T [n_cls][ncol][16][RS]: class matrices of shared local matrices (affine, p >= 3), or NULL
  const uint8_t *piv_perm; // [n_pivoting][16]: partial-pivoting row order of each solve not certified for natural-order
                           // elimination (element matrices), or NULL
  const double *geo_fd;    // double copy of geo_f
  const int32_t *nbr;      // [ne][4] neighbour or -(bf+1)
  const int8_t *nbr_face;  // [ne][4]
  const uint8_t *mask;     // [nd][ne] inflow-face bits
  const double *omega;     // [nd][2]
  const double *weight;    // [nd]
  const double *sig;       // [ne][2] sigma_t, sigma_s
  const int32_t *bf_ef;    // [nbf] 4*e + f
  double *bnd;             // [nbf][nq][2] boundary sums of the last sweep
  const double *tab_d;     // double tables of (p, nq): V, Dx, Dy [Q][n] then F [nq][p+1]
  const int32_t *dir_group;   // [nd] direction class
  const int32_t *n_levels_g;  // [n_groups] levels per class
  const int32_t *level_off;   // [n_groups][n_levels + 1] offsets into order
  const int32_t *order;       // [n_groups][ne] elements by (level, id)
  const int2 *desc_ef;        // [n_groups][ne] in order: (element, inflow mask | neighbour faces << 4)
  const int4 *desc_nb;        // [n_groups][ne] in order: neighbours (or -(boundary face + 1))
  const uint32_t *desc_up;    // [n_groups][ne][4] in order: upwind level gap | position << 8 | face << 30
  int n_levels, n_groups;
};

// Per-problem buffers of one run.
struct KIO {
  const double *phi_in;
  const double *q_iso;
  const double *q_dir;
  const double *psi_bc;
  double *mom;
  void *psi;      // T [nd][ne][n]
  double *resid;  // [n_iter] (library scratch when the caller passes NULL)
};

struct KMomIO {
  const double *mom, *q_iso, *q_dir, *psi_bc;
  double *E, *Eb, *Jin, *Q0, *Q1;
  int *n_nonpos;
};

// Launch helpers (defined in kernels.hip).  All return the launch's hipError_t.
// One sweep launch (both schedules).
struct SweepLaunch {
  int p, nq;
  bool fp32;
  int mode;          // 0: general elements, pivoting; 1: general, pivot-free; 2: affine, pivot-free
  const int4 *desc;  // level schedule: two records per entry of list (element, direction | problem << 16,
                     // flags, w), (neighbours); flags as the kernels' SolveIn flags, boundary faces << 16;
                     // w: class of shared local matrices, or entry of KProb::piv_perm; persistent
                     // schedule: the records of the whole solve list, which the tasks index
  const int2 *list;  // level schedule: (element, direction | problem << 16) pairs of one level;
                     // direction-resident schedule: (problem, direction) tasks
  int count;       // level: solves; direction-resident: tasks; persistent: tasks
  int width;       // direction-resident: widest upwind level
  int max_levels;  // direction-resident: deepest level count (offsets staged in LDS)
  int max_gap;     // pipelined: largest level gap of an upwind edge that is not lagged
  int waves;       // pipelined: waves per work-group (0 = default)
  int ring;        // pipelined: trace ring depth in levels (0 = default)
  int fixup;       // 1: negative-flux fixup after each local solve (kernel variant)
  long long wait_spins;   // pipelined: bound of a wait, in polls of about 64 clocks each
  bool flow;             // persistent schedule: list = every solve of the handle in level order
  const int2 *tasks;     // persistent: (first solve, solves) of this variant's tasks
  const int *pred_ptr;   // persistent: [count + 1] offsets into pred_idx
  const int *pred_idx;   // persistent: flag indices of each task's predecessor tasks
  int *flags;            // persistent: per task of the handle, sweep number when done (zeroed by each run)
  int own_base;          // persistent: flag index of this variant's first task
  int *abort_flag;       // persistent: set when a wait expires (zeroed by each run)
  int n_cu;              // persistent and streaming level launches: compute units of the device
  bool single;           // the handle holds one problem (streaming level kernels)
  bool shared;           // row-set LU level launches solve with the class matrices (KProb::cls_inv; one
                         // problem, streaming form; the fourth descriptor field is the class)
  const KProb *probs;
  const KIO *io;
  const void *tables;
  const void *tables_g;  // general-element tables (the pipelined kernel on general elements)
  int it;
  const int *stop;
  int *status;
  int block;
  size_t lds_max;
  hipStream_t stream;
};

hipError_t launch_sweep_level(const SweepLaunch &L);
hipError_t launch_sweep_dir(const SweepLaunch &L);
// nd: the problem's directions (1..1024), the size of the staged direction
// table.
hipError_t launch_moments(bool fp32, const KProb *probs, const KIO *io, int prob, int ne_n, int nd, int it,
                          const int *stop, hipStream_t s);
hipError_t launch_boundary(bool fp32, const KProb *probs, const KIO *io, int prob, int nbf, int nq,
                           int p, const int *stop, hipStream_t s);
hipError_t launch_run_init(const KIO *io, int n_probs, int n_iter, int *stop, int *iters, int *status,
                           hipStream_t s);
// Zero n ints (counters of the persistent schedule) with a kernel, not a
// memset node, so that a captured run replays correctly.
hipError_t launch_zero_ints(int *p, int n, hipStream_t s);
hipError_t launch_finalize(const KIO *io, int n_probs, int it, double tol, int *stop, int *iters,
                           int *iters_user, hipStream_t s);
hipError_t launch_closures(const KProb *probs, const KMomIO *io, int prob, int ne, int Q, int n, int nbf,
                           int nq, hipStream_t s);
hipError_t launch_zero_nonpos(const KMomIO *io, int n_probs, hipStream_t s);

// Direction-independent element matrices of general elements of degree 3
// (emat.hip): M, G^x, G^y [n][n] and the face matrices [4][2][p+1][p+1] of
// each element from the double volume geometry geo_vd [ne][Q][5] (w J,
// w adj(F)), the double face geometry geo_fd [ne][4][nq][2] and the double
// tables of (p, nq); written in float or double.
hipError_t launch_elem_mat(int p, int nq, bool fp32, int ne, const double *tab_d, const double *geo_vd,
                           const double *geo_fd, void *out, hipStream_t s);

// Matrices of classes of solves that share their local matrix (row-set LU
// kernels, affine elements, p >= 3): for each class c, with the local matrix
// A of its representative (element, direction, inflow faces) rep[c] = (e, d,
// inflow, 0) of problem 0, K = A^-1 R, where R maps a solve's inputs (nodal
// source [n], interior-face traces [4][tw], boundary data [4][tw], q_dir [Q];
// tw = max(p + 1, nq)) to its right-hand side; formed in double
// (Gauss-Jordan, partial pivoting on [A | R]) and written as T
// out[c][ncol][16][RS], ncol = n + 8 tw + Q, entry [j][r][s] = K[r + s H][j]
// (zero where r + s H is not a row), the slot layout of the row-set LU.  A
// zero pivot sets bit 0 of *status.
struct ClassInvLaunch {
  int p, nq;
  bool fp32;
  int n_cls;
  const int4 *rep;
  const KProb *probs;
  const void *tables;  // affine table blob of (p, nq)
  void *out;
  int *status;
  hipStream_t stream;
};
hipError_t launch_class_inv(const ClassInvLaunch &L);

// Row orders of partial pivoting for the local matrices of general elements
// (p = 3, element matrices) not certified for elimination in natural order:
// list[i] = (element, direction) of problem `prob`; out[16 i + k] = the row
// that is the pivot of elimination step k.  Reads probs[prob].emat, mask,
// omega and sig.
struct PivotOrderLaunch {
  int p;
  bool fp32;
  int n;
  const int2 *list;
  const KProb *probs;
  int prob;
  uint8_t *out;
  hipStream_t stream;
};
hipError_t launch_pivot_order(const PivotOrderLaunch &L);

// Element-local HRT VEF blocks and their inverse (hrt.hip), affine elements.
struct HrtLaunch {
  int p, nq, ne;
  const double *tab;   // vefplan::build_hrt_tables blob
  const double *geo;   // [ne][13]: J, adj(F) row major, face chords N_0..N_3
  const double *sig;   // [ne][2]: sigma_t, sigma_s
  const int32_t *nbr;  // [ne][4]: neighbour or -(boundary face + 1)
  const double *mom;   // [6][ne][(p+1)^2] transport moments
  const double *Eb;    // [nbf][nq] or NULL
  double *out;         // [ne][n][n]
  hipStream_t stream;
};
hipError_t launch_hrt_inverse(const HrtLaunch &L);

// Element-local part of the hybridized solve (couplings to the face
// multipliers, right-hand sides, the element's H and r contributions and the
// pieces of its recovery), from the block inverses of launch_hrt_inverse.
struct HrtReduceLaunch {
  int p, nq, ne;
  const double *tab, *geo;
  const int32_t *nbr;
  const int8_t *nbr_face;
  const double *mom, *Eb, *Jin, *Q0, *Q1, *inv;
  double *hloc, *rloc, *sol0, *resp;
  hipStream_t stream;
};
hipError_t launch_hrt_reduce(const HrtReduceLaunch &L);

}  // namespace vefk
