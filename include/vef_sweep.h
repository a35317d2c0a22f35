/*
 * vef_sweep.h -- C ABI of the MI355X (gfx950) discrete-ordinates DG transport
 * sweep and VEF-moment library.
 *
 * What it computes.  For the steady, mono-energetic transport equation with
 * isotropic scattering (Olivier & Haut, "High-Order Mixed Finite Element
 * Variable Eddington Factor Methods", Sec. 2, Eq. eq:transport with inflow
 * condition eq:trans_bc), discretised in angle by discrete ordinates and in
 * space by an upwind discontinuous Galerkin method of degree p on curved
 * quadrilateral meshes (Sec. 5; meshes and reference-space integration of
 * Sec. 3.1-3.2; DG space Y_p of Sec. 4.1):
 *   - vef_sweep_run: for every direction and every element, in upwind order,
 *     assemble the (p+1)^2-unknown local system by quadrature and solve it
 *     (a transport sweep), then reduce the angular flux to its angular moments
 *     phi, J, P (the numerator and denominator sums of Eq. eq:vef_disc);
 *     optionally repeat as a source iteration with the max-norm residual of
 *     successive scalar-flux iterates (stopping rule of Sec. 8);
 *   - vef_moments: the VEF closures at quadrature points: the Eddington
 *     tensor E = P/phi (ratio of DG functions, Sec. 5), the boundary factor
 *     E_b (Eq. eq:vef_disc), the inflow partial current J_in and the source
 *     moments Q_0, Q_1 (Sec. 2).
 *
 * Discretisation conventions (fixed by this library, and identical in its
 * test oracle):
 *   - reference element [0,1]^2, coordinates (xi, eta); element map of order
 *     m from (m+1)^2 control points at Gauss-Lobatto points, xi fastest;
 *   - angular flux basis: tensor Lagrange polynomials through the p+1
 *     Gauss-Lobatto points, node index a + (p+1) b (a along xi);
 *   - quadrature: tensor Gauss-Legendre, nq points per direction
 *     (default p + m), volume point index qx + nq*qy, ascending;
 *   - faces 0: eta=0, 1: xi=1, 2: eta=1, 3: xi=0, each parameterised
 *     counter-clockwise by s in [0,1]; face points ascending in s;
 *   - the upwind side of a face is chosen for the whole face from the sign
 *     of Omega . N_F, N_F the clockwise-rotated chord from the face's first
 *     to its last corner (equal to the integral of n ds); a zero product makes
 *     the lower element id upwind; a boundary face is inflow when
 *     Omega . N_F < 0;
 *   - boundary faces are numbered in ascending (element, local face) order.
 *
 * Errors: every call returns a status (VEF_OK or a negative VEF_ERR_*).
 * vef_last_error(h) returns a message for the last failure on h, or for the
 * last failed create when h is NULL.  Handles are not thread-safe; calls on
 * one handle must not overlap.
 */
#ifndef VEF_SWEEP_H
#define VEF_SWEEP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vef_sweep vef_sweep_t;

enum {
  VEF_OK = 0,
  VEF_ERR_INVALID = -1,  /* bad argument, size or mesh */
  VEF_ERR_CYCLE = -2,    /* upwind graph of some direction is cyclic (and
                            vef_options.cycles is VEF_CYCLES_REJECT) */
  VEF_ERR_JACOBIAN = -3, /* element map with J <= 0 at a quadrature point */
  VEF_ERR_HIP = -4,      /* HIP runtime failure (no device, launch error) */
  VEF_ERR_OOM = -5,      /* device or host allocation failed */
  VEF_ERR_TIMEOUT = -6   /* a bounded device-side wait of a sweep kernel
                            expired (vef_sweep_check; bound set by
                            vef_options.wait_polls) */
};

enum { VEF_FP64 = 0, VEF_FP32_LOCAL = 1 };
enum {
  VEF_CYCLES_REJECT = 0, /* a cyclic upwind graph fails with VEF_ERR_CYCLE */
  VEF_CYCLES_LAG = 1     /* a cyclic upwind graph is swept with lagged
                            couplings (vef_options.cycles) */
};
enum {
  VEF_UPWIND_FACE = 0,  /* one upwind side per face, from the rotated chord */
  VEF_UPWIND_POINT = 1  /* the upwind side at each face quadrature point
                           (vef_options.upwind) */
};
enum {
  VEF_SCHEDULE_AUTO = 0, /* VEF_DIR_RESIDENT when every problem's mean level
                            width fits one round of a work-group, else
                            VEF_LEVEL_SYNC */
  VEF_LEVEL_SYNC = 1,    /* one launch per upwind level over all directions */
  VEF_DIR_RESIDENT = 2,  /* one launch per sweep; one work-group per (problem,
                            direction) walks all upwind levels with work-group
                            barriers between levels */
  VEF_PERSISTENT = 3     /* one launch per sweep and kernel variant: every
                            resident wave takes tasks of consecutive solves
                            in upwind-level order and waits on dependency
                            counters in global memory (agent-scope
                            release/acquire, bounded by
                            vef_options.wait_polls); variants without a
                            persistent kernel (affine p <= 2, the fixup)
                            run level-synchronously */
};

/* One transport problem (host pointers, copied by vef_sweep_create and not
 * retained).  Mirrors the problem statement of Sec. 2 (sigma_t, sigma_s),
 * the mesh description of Sec. 3.1 (control points + local nodal map), the
 * degree p of Y_p (Sec. 4.1) and the discrete-ordinates set of Sec. 5. */
typedef struct {
  int p;                  /* DG degree, 1..4 */
  int m;                  /* geometry order, 1..3 */
  int nq;                 /* Gauss points per direction; 0 = p + m; else p+1..p+3 */
  int n_elem;             /* elements, 1..4194304 */
  int n_cp;               /* control points, >= 4 */
  const double *cp_xy;    /* [n_cp][2] */
  const int32_t *elem_cp; /* [n_elem][(m+1)^2] control point ids, xi fastest */
  int n_dir;              /* directions, 1..1024 */
  const double *omega;    /* [n_dir][2] in-plane components, |Omega| <= 1 */
  const double *weight;   /* [n_dir] positive, sum 4 pi (checked to 1e-12 rel) */
  const double *sigma_t;  /* [n_elem] total cross section, >= 0 */
  const double *sigma_s;  /* [n_elem] scattering cross section, >= 0 */
} vef_problem_desc;

typedef struct {
  int precision; /* VEF_FP64: every step in double.  VEF_FP32_LOCAL: local
                    assembly and solves in float with float accumulation,
                    angular flux stored as float; moments, residual and
                    closures in double. */
  int schedule;  /* VEF_SCHEDULE_AUTO, VEF_LEVEL_SYNC, VEF_DIR_RESIDENT or
                    VEF_PERSISTENT */
  int block;     /* work-group size for the sweep kernels; 0 = default 256 */
  int timing;    /* k > 0: runs record HIP events around the sweep kernels
                    of every k-th source iteration and of the last one (read
                    with vef_sweep_timing); 1 = every iteration; 0 = off.
                    Each event costs a few microseconds of device time */
  int pipeline_waves; /* waves per work-group of the pipelined
                    direction-resident kernel (affine elements, p <= 2):
                    0 = default 8, 1..8; -1 = use the row-per-lane
                    kernel instead) */
  int pipeline_ring;  /* levels of face traces the pipelined kernel keeps in
                    LDS (0 = default 4; 1..4, rounded down to a power of
                    two; fewer when LDS is short);
                    upwind elements further back are read from the angular
                    flux in global memory */
  int fixup;         /* 1: negative-flux fixup after each local solve: when an
                    element's solution has a negative nodal value, negatives
                    become zero and the rest is scaled so that the element's
                    particle balance (outflow + absorption, testing with
                    u = 1) is unchanged; non-negative solutions are untouched.
                    A simpler stand-in for the paper's QP fixup (Sec. 8.4).
                    0 = off (default) */
  int cycles;        /* what a cyclic upwind graph (re-entrant faces; Sec. 8,
                    thick diffusion limit, triple-point mesh) does:
                    VEF_CYCLES_REJECT (default): create fails with
                    VEF_ERR_CYCLE.  VEF_CYCLES_LAG: the sweep lags the
                    couplings that close cycles (the strictly upper block
                    triangular part of the streaming-collision operator in
                    the sweep order).  The order per direction: Kahn's
                    algorithm on the upwind graph; whenever every element
                    left has an unsolved upwind neighbour, the one with the
                    fewest (lowest id on ties) is released, and its inflow
                    faces from unsolved neighbours become lagged.  A lagged
                    face reads the upwind element's angular flux as it was
                    before the sweep: the previous sweep of the run, and for
                    the first sweep of a run the contents of psi_out on entry
                    (zero it to start from zero), or, when psi_out is NULL,
                    the handle's own copy from the last run (zero after
                    create).  Acyclic graphs are swept exactly as with
                    VEF_CYCLES_REJECT.  The pipelined kernel is not used for a
                    problem with lagged faces. */
  int upwind;        /* VEF_UPWIND_FACE (default): the upwind side of a face is
                    chosen for the whole face from the sign of Omega . N_F,
                    N_F the rotated chord (lower element id upwind on a zero
                    product).  VEF_UPWIND_POINT: chosen at each face
                    quadrature point from the sign of Omega . n there; on a
                    curved face whose points have both signs each element
                    takes the other's trace where it is downwind, so both
                    depend on each other and the sweep needs
                    VEF_CYCLES_LAG.  Straight faces give the same result
                    under both rules.  Not combined with the fixup. */
  long long wait_polls; /* bound of one device-side wait of a sweep kernel
                    that waits for upwind work of other waves (the pipelined
                    and persistent kernels), in polls of about 64 clocks
                    each; 0 = default
                    2^26 (seconds: a healthy wait takes microseconds).  When a
                    wait exceeds it the kernel stops its sweep early, every
                    wave exits normally and vef_sweep_check reports
                    VEF_ERR_TIMEOUT (the outputs of that run are then
                    incomplete).  Small values exist to test that path. */
  int elem_matrices; /* general (curved) elements of degree 3 with the
                    whole-face upwind rule: 0 (default) = form each element's
                    direction-independent matrices (mass, the two streaming
                    matrices, face matrices) once at create, on the matrix
                    cores, and assemble each local system from them
                    (VEF_KERNEL_GENERAL_MAT); -1 = assemble every local system
                    by quadrature (VEF_KERNEL_PIVOT / VEF_KERNEL_NOPIVOT).
                    Costs 6 KB (double) or 3 KB (float) per element. */
  int shared_matrices; /* affine elements of degree 3 or 4, one problem per
                    handle: 0 (default) = where many (direction, element)
                    pairs have the same local matrix (same sigma_t, same
                    affine geometry, same direction, hence the same outflow
                    faces; a uniform grid with few materials), group them into
                    classes at create, and in every run form one matrix per
                    class before the first sweep: K = A^-1 R, R the linear
                    map from a solve's inputs (nodal source, upwind traces,
                    boundary data, q_dir) to its right-hand side (double,
                    Gauss-Jordan with partial pivoting on [A | R]); the
                    level-synchronous sweep then computes each local
                    solution as K times the solve's inputs
                    (VEF_KERNEL_AFFINE_SHARED).  Used when there are at most
                    4096 element classes, the solves number at least 8 per
                    class and the class matrices take at most 16 MiB
                    ((n + 8 max(p + 1, nq) + nq^2) x 16 x ceil(n / 16)
                    entries each).  The local systems and their right-hand
                    sides are the same; results differ from the row-set LU
                    only by rounding.
                    -1 = never (VEF_KERNEL_AFFINE_LU). */
} vef_options;

/* Per-problem device buffers of one run (device pointers owned by the caller).
 * n = (p+1)^2, Q = nq^2, n_bf = boundary faces (vef_problem_info). */
typedef struct {
  const double *phi_in; /* [n_elem][n] scalar flux for the scattering source of
                           the first sweep; NULL = 0.  Later source iterations
                           use the previous sweep's phi. */
  const double *q_iso;  /* [n_elem][n] isotropic source per steradian, nodal; NULL = 0 */
  const double *q_dir;  /* [n_dir][n_elem][Q] source at volume points; NULL = 0 */
  const double *psi_bc; /* [n_dir][n_bf][nq] inflow data at boundary points; NULL = vacuum */
  double *mom;          /* [6][n_elem][n] out: phi, Jx, Jy, Pxx, Pxy, Pyy (nodal) */
  void *psi_out;        /* [n_dir][n_elem][n] out: angular flux, double (VEF_FP64)
                           or float (VEF_FP32_LOCAL); NULL = kept internally.
                           With lagged faces (vef_options.cycles) also an
                           input: the previous iterate for the first sweep */
  double *resid;        /* [n_iter] out: max_j |phi_new_j - phi_in_j| per sweep; may be NULL */
} vef_problem_io;

typedef struct {
  const vef_problem_io *io; /* host array [n_probs] */
  int n_iter;               /* sweeps of source iteration, >= 1 */
  double tol;               /* > 0: stop (device-side test) once every problem's
                               residual is < tol; later sweeps are skipped */
  int *iters_done;          /* device int out: sweeps performed; may be NULL */
} vef_run_args;

/* Per-problem device buffers of vef_moments (device pointers, caller-owned). */
typedef struct {
  const double *mom;    /* [6][n_elem][n] from vef_sweep_run */
  const double *q_iso;  /* as in the run (for Q0, Q1); may be NULL */
  const double *q_dir;  /* as in the run; may be NULL */
  const double *psi_bc; /* as in the run (for J_in); may be NULL */
  double *E;            /* [3][n_elem][Q] out: Exx, Exy, Eyy at volume points; may be NULL */
  double *Eb;           /* [n_bf][nq] out; may be NULL */
  double *Jin;          /* [n_bf][nq] out; may be NULL */
  double *Q0;           /* [n_elem][Q] out; may be NULL */
  double *Q1;           /* [2][n_elem][Q] out; may be NULL */
  int *n_nonpos;        /* device int out: points where phi <= 0 (E left 0) plus
                           boundary points with a non-positive denominator (E_b
                           left 0); may be NULL */
} vef_moment_io;

typedef struct {
  int n;         /* unknowns per element, (p+1)^2 */
  int nq;        /* Gauss points per direction */
  int Q;         /* volume points per element */
  int n_bf;      /* boundary faces */
  int n_levels;  /* deepest upwind level over directions, plus one */
  int n_groups;  /* classes of directions sharing one upwind graph */
  int pivoting;  /* 1: local solves use partial pivoting; 0: every face is
                    straight and sigma_t > 0, so the local matrices have a
                    positive definite symmetric part and are eliminated in
                    natural order */
  int affine;    /* 1: every element map is affine (constant J and adj(F)),
                    so the local matrices are assembled from reference
                    matrices scaled by the element's J and adj(F) */
  long long n_solves; /* n_elem * n_dir */
  int schedule;  /* vef_problem_info: the handle's schedule as resolved at
                    create (VEF_LEVEL_SYNC, VEF_DIR_RESIDENT or
                    VEF_PERSISTENT);
                    vef_plan_query: VEF_SCHEDULE_AUTO */
  int kernel;    /* vef_problem_info: sweep kernel of this problem,
                    VEF_KERNEL_*; vef_plan_query: -1 */
  long long n_lagged; /* lagged (direction, element, face) couplings; 0 for
                    acyclic upwind graphs */
  long long n_pivoting; /* (direction, element) pairs whose local system is
                    solved with partial pivoting (or, with element matrices,
                    in the pivot order formed at create): those the plan cannot
                    certify for elimination in natural order (sigma_t = 0,
                    or a curved face along which Omega . n changes sign or
                    takes the other role's sign); 0 when every face is
                    straight and sigma_t > 0 */
  int n_classes;    /* vef_problem_info: classes of (direction, element)
                    pairs sharing one local matrix (vef_options.
                    shared_matrices), 0 when the problem has none;
                    vef_plan_query: those a one-problem handle created
                    with the same options would form */
} vef_info;

/* Sweep kernels (vef_info.kernel). */
#define VEF_KERNEL_PIVOT 0          /* row per lane, partial pivoting */
#define VEF_KERNEL_NOPIVOT 1        /* row per lane, natural order */
#define VEF_KERNEL_AFFINE 2         /* row per lane, reference-matrix assembly */
#define VEF_KERNEL_AFFINE_PIPELINE 3 /* element per lane, LU ahead of the
                                       upwind data (direction-resident,
                                       affine, p <= 2) */
#define VEF_KERNEL_BILINEAR_PIPELINE 4 /* the same for straight-sided
                                       bilinear elements (m = 1), volume
                                       terms by quadrature */
#define VEF_KERNEL_AFFINE_LU 5       /* affine, p >= 3: a 16-lane slot per
                                       solve holding one or two rows per
                                       lane, LU in natural order */
#define VEF_KERNEL_GENERAL_MAT 6     /* general elements, p = 3: row per lane
                                       from precomputed element matrices;
                                       LU in natural order where the plan
                                       certifies it, else partial pivoting
                                       (level-synchronous and persistent:
                                       the rows taken in the pivot order
                                       formed at create, then LU in natural
                                       order; 16 bytes per such pair) */
#define VEF_KERNEL_AFFINE_SHARED 7   /* affine, p >= 3, level-synchronous: a
                                       16-lane slot per solve; the solution
                                       is the matrix of the solve's class
                                       (A^-1 times the map from inputs to
                                       right-hand side) times its inputs */

/* Validate the problems (sizes, weights, J > 0 at every volume point, acyclic
 * upwind graphs unless opt->cycles lags them), build the sweep plan on the host and upload it to the
 * current HIP device.  Synchronous.  n_probs > 1 gives one batched handle
 * whose runs sweep all problems together.  opt may be NULL (defaults). */
int vef_sweep_create(const vef_problem_desc *probs, int n_probs, const vef_options *opt,
                     vef_sweep_t **out);

/* Enqueue n_iter sweeps (+ moments, residual, boundary sums) on stream
 * (a hipStream_t; NULL = default stream).  Asynchronous: outputs are valid
 * after the stream is synchronised.  The library keeps the boundary sums of
 * the last sweep for vef_moments.  A call whose arguments equal the previous
 * call's (on a handle created without timing) issues only kernel launches,
 * so it can be captured in a HIP graph after one eager call. */
int vef_sweep_run(vef_sweep_t *h, const vef_run_args *args, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * run as vef_sweep_run, with the same kernels and results, that calls no
 * hipMalloc, hipFree or other allocating routine.  Differences:
 *   - a problem whose io.resid is NULL gets its per-sweep residuals (used by
 *     the device-side stop test) in a static device array of the library,
 *     VEF_STATIC_RESID_MAX doubles per GPU, shared by every handle and every
 *     call on that GPU and cleared by each run before use; the run fails with
 *     VEF_ERR_INVALID when the problems with a NULL resid need more than
 *     n_iter x (their count) > VEF_STATIC_RESID_MAX doubles.  Calls that
 *     overlap on one GPU (other streams, other threads) race on that array;
 *   - io.psi_out may be NULL only for a problem whose handle already holds its
 *     own angular flux (a problem with lagged couplings, or after an earlier
 *     vef_sweep_run with psi_out NULL); otherwise VEF_ERR_INVALID;
 *   - no timing events are recorded (vef_options.timing is ignored).
 * The static array's device address is looked up once per device when the
 * first handle on that device is created. */
#define VEF_STATIC_RESID_MAX 65536
int vef_sweep_run_static(vef_sweep_t *h, const vef_run_args *args, void *stream);

/* Enqueue the closure kernels for every problem (io: host array [n_probs]),
 * reading the boundary sums of the last run on h.  A call whose pointers
 * equal the previous call's issues only kernel launches, so it can be
 * captured in a HIP graph together with vef_sweep_run. */
int vef_moments(vef_sweep_t *h, const vef_moment_io *io, void *stream);

/* Free all device and host memory of h.  NULL is a no-op. */
int vef_sweep_destroy(vef_sweep_t *h);

/* Host-only: validate one problem and build its plan without touching the
 * GPU; fills *info.  Returns the status vef_sweep_create would return for the
 * problem with options opt (NULL = defaults; only opt->cycles is read),
 * except HIP and device-memory errors. */
int vef_plan_query(const vef_problem_desc *prob, const vef_options *opt, vef_info *info);

/* Sizes of problem k of a handle. */
int vef_problem_info(const vef_sweep_t *h, int k, vef_info *info);

/* Boundary faces of problem k as (element, local face) pairs, host array
 * [n_bf][2]. */
int vef_boundary_faces(const vef_sweep_t *h, int k, int32_t *out);

/* Element-local blocks of the hybridized Raviart-Thomas VEF method and their
 * inverse (Sec. 7, "Implementation Details": Eq. eq:hyb_form and the blocks
 * W, X, Y, Z of Eq. eq:block_inv), for every element of problem k, on the
 * device, from the moments of a transport run on h.  Per element K:
 *   A_ij  = int_K sigma_t v_i . v_j dx
 *           + int_{dK cap Gamma_b} (1/E_b)(v_i . E n)(v_j . n) ds   (Eq. eq:A)
 *   G_ij  = - int_K grad v_i : E u_j dx                               (hat G)
 *   D_ij  = int_K u_i div v_j dx                                      (Eq. eq:D)
 *   Ma_ij = int_K (sigma_t - sigma_s) u_i u_j dx                      (Eq. eq:Ma)
 * with v_i the RT_p basis of D_p(K) (reference Q_{p+1,p} x Q_{p,p+1} under
 * the contravariant Piola map, Eq. eq:piola; nodal at Gauss-Lobatto points
 * along the component's direction and Gauss-Legendre points across it;
 * xi-component functions first, node a + (p+2) b, then eta-component
 * functions, node a + (p+1) b) and u_i the Lagrange basis of Q_p through the
 * tensor Gauss-Legendre points (node a + (p+1) b).  E = P / phi at each
 * quadrature point from mom (the isotropic I/3 where phi <= 0).  inv receives
 * [[W, X], [Y, Z]] = [[A, G], [D, Ma]]^{-1}.
 *   mom  device [6][n_elem][(p+1)^2]: moments of vef_sweep_run;
 *   Eb   device [n_bf][nq]: E_b of vef_moments (values <= 0 taken as 1/2),
 *        or NULL (1/2 everywhere);
 *   inv  device out [n_elem][n][n] row major, n = 2(p+1)(p+2) + (p+1)^2.
 * The inverse is formed by elimination in natural order (current unknowns
 * first, then the Schur complement S = Ma - D A^{-1} G): like the block
 * formulas, it assumes A and S non-singular (sigma_t > 0) and allows a
 * singular Ma.  Quadrature: the handle's nq Gauss points per direction, which
 * must be p + 2 or p + 3 (exact for the RT mass).  Requirements: every
 * element map affine (vef_info.affine), p <= 3.  Asynchronous on stream; the
 * first call for a problem uploads its geometry and tables (synchronous).
 * Errors: VEF_ERR_INVALID (problem not affine, p or nq out of range, NULL
 * pointers), VEF_ERR_HIP, VEF_ERR_OOM. */
int vef_hrt_local_inverse(vef_sweep_t *h, int k, const double *mom, const double *Eb, double *inv,
                          void *stream);

/* Element-local part of the hybridized solve (Sec. 7, "Implementation
 * Details": the reduced system H lambda = r for the face multipliers and the
 * element-by-element recovery), for every element of problem k, on the
 * device.  With the interior-face multiplier mu (Lagrange of degree p through
 * the Gauss-Legendre points of the face, in the counter-clockwise parameter
 * of its lower-numbered element) and per element K, slot s = (f, t) for node
 * t of local face f:
 *   C1[s][i] = int_F mu_t (v_i . n) ds,  C2[i][s] = int_F (v_i . <E n>) mu_t ds
 *   (interior faces; <E n> the average of E n over the face's two sides, E =
 *   P / phi from mom; zero on boundary faces),
 *   g_i = int_K v_i . Q1 dx + sum over boundary faces
 *         2 int_F (1/E_b)(v_i . E n) J_in ds,   f_j = int_K u_j Q0 dx
 * (bases as vef_hrt_local_inverse) and, from inv = [[W, X], [Y, Z]]:
 *   sol0 = inv [g; f],   resp = inv [C2; 0],
 *   hloc = C1 W C2,   rloc = C1 (W g + X f),
 * so that H = sum_K hloc, r = sum_K rloc (assembled by slot) and the
 * element's [J; phi] = sol0 - resp lambda_K.
 *   mom  device [6][n_elem][(p+1)^2]: moments of vef_sweep_run;
 *   Eb, Jin, Q0, Q1  device: closures of vef_moments ([n_bf][nq], [n_bf][nq],
 *        [n_elem][nq^2], [2][n_elem][nq^2]); Eb may be NULL (1/2);
 *   inv  device [n_elem][n][n]: block inverses of vef_hrt_local_inverse;
 *   hloc device out [n_elem][4(p+1)][4(p+1)], rloc [n_elem][4(p+1)],
 *   sol0 device out [n_elem][n], resp [n_elem][n][4(p+1)].
 * Requirements, asynchrony and errors as vef_hrt_local_inverse (Jin, Q0, Q1,
 * inv and the outputs must not be NULL). */
int vef_hrt_reduce(vef_sweep_t *h, int k, const double *mom, const double *Eb, const double *Jin,
                   const double *Q0, const double *Q1, const double *inv, double *hloc, double *rloc,
                   double *sol0, double *resp, void *stream);

/* Device solver of the reduced hybridized system of Sec. 7 (the face
 * unknowns lambda of Eq. eq:hyb_form once every element's [J; phi] has been
 * eliminated, as vef_hrt_reduce leaves them): H lambda = r, H and r the sums
 * of the element contributions hloc, rloc over the interior-face slots of
 * each element, then [J; phi]_K = sol0_K - resp_K lambda_K per element.
 * The sparsity pattern of H is fixed by the mesh, so a host factorisation
 * P H0 Q = L U of one matrix of that pattern (for instance SuperLU's, with
 * its fill-reducing column order) is re-used: each solve re-factorises the
 * new values numerically with that pivot order and fill (rocSOLVER csrrf)
 * and solves on the device.  The re-used pivot order is only as good as it
 * is for the new matrix: the backward error returned by vef_lambda_solve
 * tells the caller when to factorise on the host again.
 *
 * vef_lambda_create arguments (host arrays unless stated):
 *   n        unknowns (interior faces x (p+1)); ne elements; k = 4(p+1)
 *            slots per element; nloc = local unknowns of [J; phi];
 *   gidx     [ne][k] unknown of each slot (face f, point t at f(p+1)+t),
 *            -1 for slots on the boundary; an unknown belongs to at most
 *            two elements;
 *   nnz_t, ptr_t [n+1], ind_t [nnz_t], val_t [nnz_t]: the factors as one CSR
 *            matrix T = (L - I) + U (unit diagonal of L not stored, columns
 *            ascending in each row) of P H0 Q = L U;
 *   piv_p, piv_q [n]: row piv_p[i] of H0 is row i of P H0, column piv_q[j]
 *            of H0 is column j of H0 Q (permutations of 0..n-1);
 *   hloc0, rloc0 (device): the element contributions of H0 and of one r,
 *            laid out as for vef_lambda_solve;
 *   stream   where the set-up runs (blocking);
 *   *out     the handle (vef_lambda_destroy frees it).
 * vef_lambda_solve arguments (device arrays):
 *   hloc [ne][k][k], rloc [ne][k]: this matrix and right-hand side;
 *   lam [n] out: the solution lambda;
 *   sol0 [ne][nloc], resp [ne][nloc][k], sol [ne][nloc] out: the recovery
 *            (all three NULL to skip it);
 *   rel_resid (host, may be NULL): the normwise backward error
 *            |r - H lambda|_inf / (|H|_inf |lambda|_inf + |r|_inf)
 *            (the call then blocks until it is known);
 *   stream   where it runs (asynchronous when rel_resid is NULL).
 * Errors: VEF_ERR_INVALID (sizes, NULL, gidx out of range, T not a sorted
 * CSR pattern, pivots not permutations), VEF_ERR_OOM, VEF_ERR_HIP (a HIP,
 * rocBLAS or rocSOLVER call failed).  vef_lambda_error gives the message
 * (h NULL: the last failed create). */
typedef struct vef_lambda vef_lambda_t;
int vef_lambda_create(int n, int ne, int k, int nloc, const int32_t *gidx, int nnz_t, const int32_t *ptr_t,
                      const int32_t *ind_t, const double *val_t, const int32_t *piv_p, const int32_t *piv_q,
                      const double *hloc0, const double *rloc0, void *stream, vef_lambda_t **out);
int vef_lambda_solve(vef_lambda_t *h, const double *hloc, const double *rloc, const double *sol0, const double *resp,
                     double *lam, double *sol, double *rel_resid, void *stream);
int vef_lambda_destroy(vef_lambda_t *h);
const char *vef_lambda_error(const vef_lambda_t *h);

/* Measured machine figures (vef_probe_machine). */
typedef struct {
  int compute_units;      /* of the current device */
  double hbm_copy_gbs;    /* device-to-device copy of 512 MiB, bytes read + written per second / 1e9 */
  double fp64_fma_tflops; /* FP64 vector FMA rate over all compute units */
  double fp32_fma_tflops; /* FP32 vector FMA rate, non-packed forms (as the library is built) */
  double lds_handoff_ns;  /* one hand-off between two waves of a work-group through an LDS counter */
} vef_machine;

/* Roofline denominators of the sweep measured on the current device, which
 * the paper does not give (a property of the machine, not of the method):
 * HBM copy rate, FP64 and FP32 vector FMA rates, and the latency of the
 * LDS-counter hand-off the pipelined sweep uses between levels.  Allocates
 * and frees about 1 GiB of device memory; blocking (runs on stream).
 * Errors: VEF_ERR_INVALID (out NULL), VEF_ERR_OOM, VEF_ERR_HIP, VEF_ERR_TIMEOUT
 * (a bounded hand-off wait expired). */
int vef_probe_machine(vef_machine *out, void *stream);

/* Result of vef_sweep_autotune. */
typedef struct {
  int schedule;       /* chosen: VEF_LEVEL_SYNC, VEF_DIR_RESIDENT or VEF_PERSISTENT */
  int pipeline_waves; /* chosen waves of the pipelined kernel; -1 = row-per-lane kernel */
  int block;          /* chosen work-group size of the level-synchronous kernels */
  int elem_matrices;  /* for problems built with element matrices (vef_options.
                         elem_matrices): 1 = the element-matrix kernel was
                         chosen, 0 = the quadrature kernel; -1 = no such problem */
  int shared_matrices; /* for a problem with classes of shared local matrices
                         (vef_info.n_classes > 0): 1 = solves by the class
                         matrices were chosen, 0 = the row-set LU; -1 = no
                         such problem */
  int n_candidates;   /* configurations timed */
  double best_ms;     /* one run of the given arguments with the choice (mean of reps) */
  double before_ms;   /* the same with the configuration the handle had before */
} vef_tune_result;

/* Same operation as vef_sweep_run (the sweep of Sec. 5 with the moments of
 * Eq. eq:vef_disc), run repeatedly to choose how it is scheduled: the
 * level-synchronous kernels with 128 or 256 threads per work-group, the
 * direction-resident row-per-lane kernel, the persistent schedule (when some
 * variant has a persistent kernel) and (when some problem has affine
 * elements of degree <= 2) the pipelined kernel with 8, 6 or 4 waves; where
 * a problem was built with element matrices (Sec. 3.2, formed on the matrix
 * cores), each schedule also with the quadrature-assembly kernel instead;
 * where a problem has classes of shared local matrices, the level-synchronous
 * kernels also with the row-set LU instead of the class matrices.  Each
 * candidate runs once untimed and then reps (1..1000) times between HIP
 * events on stream; the fastest is kept by the handle for later runs when it
 * beats the handle's configuration before the call by more than 2% (else
 * that one stays; results differ between kernels only by rounding).  Blocking.  The output
 * buffers of a hold the last candidate's results.  out may be NULL.  Errors:
 * as vef_sweep_run and vef_sweep_check; the handle then keeps its previous
 * configuration. */
int vef_sweep_autotune(vef_sweep_t *h, const vef_run_args *a, void *stream, int reps, vef_tune_result *out);

/* Synchronise the handle's last stream and return the device status word of
 * the last run (each run clears it when it starts): VEF_OK; VEF_ERR_INVALID
 * when a local solve produced a non-finite unknown (singular or overflowing
 * local system), or, as an internal error, when a level-synchronous kernel met
 * a solve list that breaks its layout (a wave with solves of two problems);
 * VEF_ERR_TIMEOUT when a bounded device-side wait of a sweep
 * kernel expired (vef_options.wait_polls; the kernel then exits without
 * finishing the sweep). */
int vef_sweep_check(vef_sweep_t *h);

/* Timing of the last run on a handle created with opt->timing != 0:
 * synchronises, then returns in *sweep_ms the summed device time from the
 * first to the last sweep kernel of each timed source iteration (HIP events
 * on the run's stream; see vef_options.timing) and in *n_launches the number
 * of sweep-kernel launches that time covers.  Either pointer may be NULL. */
int vef_sweep_timing(vef_sweep_t *h, double *sweep_ms, int *n_launches);

const char *vef_last_error(const vef_sweep_t *h);
const char *vef_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* VEF_SWEEP_H */
