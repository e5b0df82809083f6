/*
 * ppmpm.h -- C ABI of libppmpm.so: the per-step hot path of the stabilized implicit material
 * point method for coupled large-deformation poromechanics (Zhao & Choo, arXiv 1905.00671),
 * on one AMD Instinct MI355X (gfx950).
 *
 * The calls follow the problem statement of Sec. 2.4 (given boundary data u^, t^, p^, q^ and
 * initial u0, p0, find u and p) and the four-stage MPM step of Sec. 3.1: material points, a
 * fixed background grid, boundary conditions and a time step go in; the updated material-point
 * state comes out.
 *
 * Conventions shared by every call
 *   - Every function returns a ppmpm_status; ppmpm_last_error() returns a thread-local message
 *     describing the last failure.  No C++ exception or ownership crosses the ABI.
 *   - dim is 2 (plane strain) or 3.  Grid nodes are numbered ix + nx1*(iy + ny1*iz) with
 *     nx1 = ncell[0] + 1 etc. ("natural order").  Particle arrays are row-major: x[np*dim],
 *     F[np*dim*dim], ... in the caller's particle order, which the library preserves on output
 *     (it sorts particles internally).
 *   - `where` = PPMPM_HOST or PPMPM_DEVICE says whether a caller pointer is host memory or
 *     device memory of the problem's GPU.  The caller owns every array it passes; the library
 *     copies inputs into its workspace and never frees caller memory.
 *   - All device work is enqueued on the caller's HIP stream (hipStream_t passed as void*);
 *     ppmpm_step_batched also runs kernel-variant groups on streams of its own (see there).
 *     ppmpm_step returns after its statistics are available (it synchronizes the stream once
 *     per Newton iteration and a few times per Krylov solve).
 *   - A problem is not thread-safe.  Problems stepped together by ppmpm_step_batched must share
 *     the stream of the first problem of the batch.
 */
#ifndef PPMPM_H
#define PPMPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ppmpm_problem ppmpm_problem; /* opaque */

typedef enum {
    PPMPM_OK = 0,
    PPMPM_E_INVALID = 1,     /* bad argument, unsupported combination, wrong call order */
    PPMPM_E_OOM = 2,         /* workspace smaller than ppmpm_workspace_bytes */
    PPMPM_E_DEVICE = 3,      /* a HIP runtime call failed */
    PPMPM_E_NEWTON = 4,      /* Newton did not converge within newton_max iterations */
    PPMPM_E_KRYLOV = 5,      /* Krylov breakdown (reported in the statistics, not fatal) */
    PPMPM_E_NONFINITE = 6,   /* non-finite residual or an inverted material point (det dF <= 0) */
    PPMPM_E_OUT_OF_GRID = 7  /* a material point left the background grid */
} ppmpm_status;

enum { PPMPM_HOST = 0, PPMPM_DEVICE = 1 };
enum { PPMPM_LINEAR = 0, PPMPM_GIMP = 1 };              /* basis, Sec. 3.1 */
enum { PPMPM_HENCKY = 0, PPMPM_NEO_HOOKEAN = 1 };       /* skeleton, Sec. 2.2 */
enum { PPMPM_TAU_OFF = 0, PPMPM_TAU_WHITE = 1, PPMPM_TAU_SUN = 2, PPMPM_TAU_MONFORTE = 3 }; /* Sec. 4.3 */
enum { PPMPM_FP64 = 0, PPMPM_MIXED = 1 };

/* Fixed background grid (the mesh is never moved, Sec. 3.5).  Cells are squares/cubes of edge h;
 * the grid spans origin .. origin + ncell*h on every axis. */
typedef struct {
    int dim;
    int ncell[3];
    double h;
    double origin[3];
} ppmpm_grid;

/* Constants of Sec. 2: E, nu of the skeleton (Lame parameters derived from them), intrinsic
 * permeability k and fluid viscosity mu_f (mobility k/mu_f of the Darcy law), intrinsic fluid
 * density, gravity.  model: PPMPM_HENCKY (plane strain only) or PPMPM_NEO_HOOKEAN
 * (tau' = G (b - 1) + lambda ln J 1).
 * phi0: 0 keeps k constant; in (0, 1) it is the initial porosity of the Kozeny-Carman law
 * (eq. kozeny-carman), k then being the initial permeability and the porosity that of a skeleton
 * of incompressible grains, phi = 1 - (1 - phi0)/J with J = det F, held at 1e-4 below that.
 * Other values: PPMPM_E_INVALID. */
typedef struct {
    int model;
    double E, nu, k, mu_f, rho_f;
    double g[3];
    double phi0;
    double alpha_vis;  /* Kelvin-type damping parameter (s), Sec. 2.2: sigma'_vis = alpha_vis c : sym(l),
                          c = lambda 1 (x) 1 + 2 G I (the tangent at the undeformed state); used by
                          dynamic problems only (eq. quasi-static-condition), >= 0 */
} ppmpm_material;

/* Method options.
 *   shape            PPMPM_LINEAR (original MPM) or PPMPM_GIMP (2D only)
 *   dynamic          0: quasi-static, implicit Euler (eq. implicit-euler);
 *                    1: Newmark (eq. newmark) with beta, gamma
 *   tau_kind/scale   stabilization parameter of the PPP term (eq. tau-white/sun/monforte) times scale
 *   precision        PPMPM_FP64, or PPMPM_MIXED: FP32 Jacobian, SpMV, preconditioner and Krylov
 *                    vectors; FP64 residual, projection and Newton update
 *   newton_rtol      relative residual reduction required of each residual block (momentum,
 *                    mass; eq. newton-tolerance applied block-wise); newton_atol_u/p are
 *                    absolute floors (<= 0: 1e-12 E h^(dim-1) and 1e-12 h^dim/dt)
 *   newton_max       Newton iterations before PPMPM_E_NEWTON
 *   krylov_rtol      BiCGStab stops at ||r|| <= krylov_rtol ||R^k||; krylov_max caps iterations
 *   krylov_check     iterations between host checks of the convergence flag (>= 1)
 *   mg_smooth        pre/post smoothing sweeps of each multigrid V-cycle (>= 1)
 *   consistent_mass  1: Stage 1 maps p (and v, a, pdot, pddot on dynamic steps) with the consistent
 *                    mass matrix (eq. map-from-particles-to-nodes-consistent, used by the paper for
 *                    cyclic loading, Sec. 5.2): sum_j M_ij f_j = sum_mp S_i m f_mp, M_ij = sum_mp
 *                    S_i S_j m, solved by conjugate gradients to 1e-13 relative residual.  Nodes
 *                    whose lumped mass is below 1e-2 of the problem's largest nodal mass keep the
 *                    lumped value (the consistent matrix is singular in the limit of nodes that a
 *                    point domain barely reaches).  Costs a stream synchronization every 8
 *                    iterations; more workspace (ppmpm_workspace_bytes).  0: lumped (default)
 *   drained_surface  1: zero pore pressure on the current free surface of the material (Sec. 5.3:
 *                    a drained top that follows the settling material), imposed at the start
 *                    of every step on the active nodes that have an inactive node among their
 *                    3^dim - 1 neighbours inside the grid (the grid edges are supports or
 *                    symmetry planes, not free surfaces); 0: boundary data only
 *   negligible_mass  a node whose lumped mass is below this fraction of the step's largest nodal
 *                    mass is outside the material (mass, mapped fields and dofs dropped); <= 0:
 *                    1e-15.  Larger values (1e-6 for bodies in contact) drop nodes that a point
 *                    domain barely reaches, whose displacement is otherwise nearly undetermined
 *   schur            Schur-block approximation of the preconditioner (Sec. 3.4: the Schur
 *                    complement S = C - B2 A^-1 B1 is preconditioned first).  0: fixed-stress form
 *                    C + C_stab + (c_t/K) M_p, the pressure block plus a lumped storage term
 *                    (default).  1: diagonal-inverse form C - B2 diag(A)^-1 B1, diag(A) the dim x dim
 *                    node blocks of the displacement block, the product kept on the Jacobian's
 *                    stencil (exact where the pressure-displacement couplings reach one node
 *                    spacing and the stencil two, as with GIMP), with a full multigrid hierarchy.
 *                    It suits undrained dynamic problems, whose displacement block is dominated by
 *                    inertia so that S is close to a pressure Laplacian that a diagonal term
 *                    cannot represent.  One more level-0 operator in the workspace (S Nnode
 *                    entries)
 */
typedef struct {
    int shape;
    int dynamic;
    double beta, gamma;
    int tau_kind;
    double tau_scale;
    int precision;
    double newton_rtol, newton_atol_u, newton_atol_p;
    int newton_max;
    double krylov_rtol;
    int krylov_max;
    int krylov_check;
    int mg_smooth;
    int drained_surface;
    int consistent_mass;
    double negligible_mass;
    int schur;
} ppmpm_options;

/* Boundary data of one step on the grid nodes (natural order).
 *   u_fixed[nnode*dim] (0/1)  Dirichlet displacement components; u_inc their prescribed
 *                             increment over the step (the grid unknown is the incremental
 *                             displacement, the grid being reset every step, Sec. 3.1)
 *   p_fixed[nnode], p_val     Dirichlet pore pressure p^ at the end of the step
 *   f_ext[nnode*dim]          nodal external forces (integrated traction t^)
 *   q_ext[nnode]              nodal inflow (integrated flux q^ = -n.q)
 *   point_force[np*dim]       forces carried by material points (traction times the point's share
 *                             of the loaded boundary; caller's point order), for Neumann loads
 *                             that follow the material (Sec. 5.2): the force acts on the face of
 *                             the point's domain whose outward normal is point_normal (a
 *                             coordinate axis, +-1 in one component); along that axis the grid's
 *                             linear hat is evaluated on the face x_a + lp_a n_a, along the other
 *                             axes the point's own basis (hat or GIMP) distributes it.  The nodal
 *                             forces of the loaded points are added with atomics (sums in
 *                             nondeterministic order, rounding-level differences only)
 *   point_normal[np*dim]      NULL or a zero row: the force acts through the point's own basis
 *   point_p_fixed[np] (0/1), point_p_val[np]   pore pressure conditions carried by material
 *                             points (caller's order; Sec. 5.4 drains the bodies through a few
 *                             points): every active node in the basis of a flagged point holds
 *                             the point's value (NULL values: 0); applied after all other
 *                             conditions of the step.  A node reached by flagged points with
 *                             different values gets one of them
 * Any pointer may be NULL (no condition / zero).  Conditions on inactive nodes are ignored; a
 * node is active when its lumped mass exceeds 1e-15 of the step's largest nodal mass (a node that
 * a point domain only just reaches is outside the material).  The point arrays are read with the
 * same `where` as the others. */
typedef struct {
    const uint8_t* u_fixed;
    const double* u_inc;
    const uint8_t* p_fixed;
    const double* p_val;
    const double* f_ext;
    const double* q_ext;
    int where;
    const double* point_force;
    const double* point_normal;
    const uint8_t* point_p_fixed;
    const double* point_p_val;
} ppmpm_bc;

#define PPMPM_MAX_HIST 64
/* Per-step statistics.  res_u/res_p: L2 norms of the momentum and mass residual blocks at each
 * Newton iteration (free degrees of freedom only); krylov_iters per Newton iteration; times in
 * seconds measured on the host around the synchronized phases.  The Jacobian and preconditioner
 * set-up (t_precond) is timed apart only while kernel timing is enabled (ppmpm_timing_enable);
 * otherwise it is part of t_krylov and t_precond is 0. */
typedef struct {
    int status;
    int newton_iters;
    int converged;
    int krylov_total;
    int krylov_iters[PPMPM_MAX_HIST];
    double res_u[PPMPM_MAX_HIST];
    double res_p[PPMPM_MAX_HIST];
    double t_sort, t_assemble, t_precond, t_krylov, t_g2p, t_total;
    int krylov_breakdowns;   /* BiCGStab breakdowns: restarted from the current residual, or ending a solve */
    int ngrid_levels;
    int mass_iters;   /* CG iterations of the consistent-mass mapping (0: lumped) */
} ppmpm_step_stats;

/* Device bytes of workspace a problem with this grid, particle count and options needs.
 * Admission control (serving) compares this against free HBM. Returns 0 on invalid input. */
size_t ppmpm_workspace_bytes(const ppmpm_grid* grid, int64_t np, const ppmpm_options* opt);

/* Creates a problem on the current HIP device.  `workspace` is caller-allocated device memory
 * of at least ppmpm_workspace_bytes bytes, 256-byte aligned, kept alive until ppmpm_destroy;
 * `hip_stream` is the stream all work of the problem is enqueued on.  The library performs no
 * device allocation of its own.  Errors: PPMPM_E_INVALID (bad sizes, GIMP in 3D, Hencky in 3D),
 * PPMPM_E_OOM (workspace too small). */
ppmpm_status ppmpm_create(const ppmpm_grid* grid, const ppmpm_material* mat,
                          const ppmpm_options* opt, void* workspace, size_t ws_bytes,
                          void* hip_stream, int64_t np, ppmpm_problem** out);

/* Initial material-point state (Sec. 2.4 initial conditions): positions x[np*dim], volumes
 * vol[np], masses mass[np], GIMP half-lengths lp[np*dim] (NULL: h/4), initial velocities
 * v0[np*dim] (NULL: 0) and pore pressures p0[np] (NULL: 0).  F = 1, u = 0.  np must equal the
 * count given to ppmpm_create.  PPMPM_E_OUT_OF_GRID if a point lies outside the grid. */
ppmpm_status ppmpm_set_particles(ppmpm_problem* p, int64_t np, const double* x, const double* vol,
                                 const double* mass, const double* lp, const double* v0,
                                 const double* p0, int where);

/* One implicit time step of length dt (Stages 1-4 of Sec. 3.1): counting sort of the points into
 * cells, lumped P2G, Newton iterations (residual and fixed-stencil block-CSR Jacobian with the
 * PPP term; BiCGStab with the block upper-triangular preconditioner), G2P update.  A Newton
 * update that inverts a material point or makes the residual non-finite is halved (up to four
 * times) before the step fails.  The step is transactional: on PPMPM_E_NEWTON, PPMPM_E_NONFINITE or PPMPM_E_OUT_OF_GRID the material-point
 * state is left unchanged and the caller may retry (e.g. with a smaller dt).  stats may be NULL. */
ppmpm_status ppmpm_step(ppmpm_problem* p, double dt, const ppmpm_bc* bc, ppmpm_step_stats* stats);

/* Steps nprob problems together: one kernel launch per phase over all problems that share a
 * kernel variant (dimension, basis, precision) and Krylov options (krylov_rtol, krylov_max,
 * krylov_check), each problem converging independently.  The groups advance in lockstep, the
 * first on the problems' stream and the others on streams the library creates (default
 * priority, kept until the process ends), so that their work overlaps on the device; the call
 * returns after all of it has completed.  dt[nprob], bcs[nprob], stats[nprob]: every
 * stats[i].status is set, also when the call fails (a problem the step did not finish carries
 * the call's failure).  A problem without particles, with dt <= 0 or on another stream than the
 * first valid problem of the batch gets PPMPM_E_INVALID and is not stepped; the others are.
 * Returns PPMPM_OK if every problem succeeded, otherwise the first failing status; a failing
 * problem does not affect the others. */
ppmpm_status ppmpm_step_batched(ppmpm_problem* const* probs, int nprob, const double* dt,
                                const ppmpm_bc* const* bcs, ppmpm_step_stats* stats);

/* Material-point fields, caller's order. */
enum {
    PPMPM_FIELD_X = 0,     /* position        [np*dim] */
    PPMPM_FIELD_U = 1,     /* displacement    [np*dim] accumulated since the start */
    PPMPM_FIELD_P = 2,     /* pore pressure   [np] */
    PPMPM_FIELD_F = 3,     /* deformation gradient [np*dim*dim] */
    PPMPM_FIELD_VOL = 4,   /* volume          [np] */
    PPMPM_FIELD_SIG = 5,   /* effective Cauchy stress [np*9] full 3x3 */
    PPMPM_FIELD_V = 6,     /* velocity        [np*dim] */
    PPMPM_FIELD_A = 7,     /* acceleration    [np*dim] */
    PPMPM_FIELD_PD = 8,    /* pdot            [np] */
    PPMPM_FIELD_PDD = 9,   /* pddot           [np] */
    PPMPM_FIELD_LP = 10    /* GIMP half-lengths [np*dim] */
};
ppmpm_status ppmpm_get_field(const ppmpm_problem* p, int field, double* out, int where);

/* Checkpoint and resume.  A problem carries nothing from one step to the next but its material
 * points: the background grid is reset every step (Sec. 3.1) and the mappings, Newton and
 * Krylov solves start afresh.  A checkpoint is therefore the committed point state: a 64-byte
 * header (the bytes "PPMPMST1", format version, dim, shape, fields per point, np, cells per axis,
 * h), every per-point field in the problem's current cell-sorted order, and the points' ids.
 *   ppmpm_state_bytes  size of a checkpoint of p
 *   ppmpm_save_state   writes it to out[bytes] (host or device memory, `where`); needs points
 *   ppmpm_load_state   restores one into p, a problem created with the same grid, material,
 *                      options and point count; steps then continue bit for bit as they would
 *                      have from the saved problem
 * PPMPM_E_INVALID for a null pointer, a buffer smaller than ppmpm_state_bytes, a problem without
 * points (save), or a header that does not match p (load); p is unchanged then.  The caller owns
 * the buffer; both calls return after the copy has completed. */
ppmpm_status ppmpm_state_bytes(const ppmpm_problem* p, size_t* bytes);
ppmpm_status ppmpm_save_state(const ppmpm_problem* p, void* out, size_t bytes, int where);
ppmpm_status ppmpm_load_state(ppmpm_problem* p, const void* in, size_t bytes, int where);

/* Inspection of one Newton iterate, for verification.  Performs Stage 1 (sort, P2G) for the
 * current state with boundary data bc and step dt, then evaluates the residual and assembles the
 * Jacobian at the nodal state U[nnode*dim], P[nnode] (natural order).  R[nnode*(dim+1)] receives
 * the residual (node-interleaved [u..., p]) with non-free degrees of freedom set to zero.  The
 * Jacobian stays in the workspace for ppmpm_apply_jacobian. */
ppmpm_status ppmpm_eval_residual(ppmpm_problem* p, double dt, const ppmpm_bc* bc, const double* U,
                                 const double* P, double* R, int where);

/* For callers that cannot allocate (code under HIP stream capture, serving loops and harnesses that
 * forbid hipMalloc): ppmpm_create + ppmpm_set_particles + ppmpm_eval_residual in one call, with
 * the problem's workspace in a device array inside the library (64 MiB per GPU, held until the
 * process ends) instead of caller memory; the call allocates nothing.  Arguments as in those
 * three calls (x, vol, mass, lp, v0, p0 the initial material points; U, P, R the nodal state
 * and the residual out; where applies to every array).  PPMPM_E_OOM when the problem needs more
 * than 64 MiB (ppmpm_workspace_bytes).  Every call on a GPU uses that GPU's array and the
 * library's host staging, which keep the last call's contents: calls that overlap (other threads,
 * other streams) race.  The call returns after its work has completed. */
ppmpm_status ppmpm_eval_residual_static(const ppmpm_grid* grid, const ppmpm_material* mat, const ppmpm_options* opt,
                                        int64_t np, const double* x, const double* vol, const double* mass,
                                        const double* lp, const double* v0, const double* p0, double dt,
                                        const ppmpm_bc* bc, const double* U, const double* P, double* R,
                                        void* hip_stream, int where);

/* y = J v with the Jacobian of the last ppmpm_eval_residual (non-free rows act as identity);
 * v, y are [nnode*(dim+1)] node-interleaved. */
ppmpm_status ppmpm_apply_jacobian(ppmpm_problem* p, const double* v, double* y, int where);

/* Nodal fields of the last Stage 1 (natural order): 0 lumped mass M, 1 P_n, 2 free-dof mask as
 * doubles [nnode*(dim+1)]; 3 the Newton iterate [U, P] (node-interleaved, [nnode*(dim+1)]) that the
 * last ppmpm_step / ppmpm_eval_residual used: after a successful step, the converged increments
 * of Sec. 3.4 that the G2P update of Sec. 3.5 consumed. */
ppmpm_status ppmpm_get_nodal(const ppmpm_problem* p, int field, double* out, int where);

ppmpm_status ppmpm_destroy(ppmpm_problem* p);
const char* ppmpm_last_error(void);

/* Kernel timing for measurement (process-wide).  When enabled, HIP events are recorded on the
 * launching stream around every launch of the kernels below; ppmpm_timing_get returns the number
 * of launches and their summed duration in milliseconds since the last reset.
 *   0 SpMV of the Krylov solver   1 Jacobian block rows   2 quadrature records   3 residual
 *   4 finest-level sweeps of the displacement-block multigrid   5 P2G   6 G2P
 *   7 sort permutation   8 Galerkin coarse operators   9 3D cell matrices (the block rows of 3D
 *   problems are then summed from them by launch 1)   10 finest-level sweeps of the Schur-block
 *   multigrid */
enum { PPMPM_K_SPMV = 0, PPMPM_K_JACOBIAN, PPMPM_K_RECORDS, PPMPM_K_RESIDUAL, PPMPM_K_MG0_RESID,
       PPMPM_K_P2G, PPMPM_K_G2P, PPMPM_K_PERMUTE, PPMPM_K_RAP, PPMPM_K_CELLMAT, PPMPM_K_MG0_S,
       PPMPM_K_COUNT };
ppmpm_status ppmpm_timing_enable(int on);
ppmpm_status ppmpm_timing_reset(void);
ppmpm_status ppmpm_timing_get(int kernel, int64_t* launches, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif
