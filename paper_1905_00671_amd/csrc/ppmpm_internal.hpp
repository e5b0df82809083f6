// Internal declarations of libppmpm: the device-side problem descriptor, memory layouts and
// the device functions shared by the kernels (basis functions of Sec. 3.1, constitutive laws of
// Sec. 2.2).  Nothing here is part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppm {

constexpr int MAXB = 64;      // problems per batched launch
constexpr int TPB = 256;      // threads per block of the streaming kernels
constexpr int MCOL = 9;       // most fields of one consistent-mass mapping (3D dynamic: 2 dim + 3)
constexpr int MAXLEV = 12;    // multigrid levels
constexpr int CMAX = 112;     // largest coarsest-level system solved by a dense inverse (LDS, 101 KB)
constexpr int TAILMAX = 200;  // levels with at most this many nodes run inside one fused kernel
// node tiles of the residual gather (RES_NODES nodes, one block of RES_PARTS wavefronts per tile)
constexpr int TILE2X = 16, TILE2Y = 4;
constexpr int TILE3X = 8, TILE3Y = 8, TILE3Z = 1;
constexpr int RES_NODES = 64, RES_PARTS = 4;  // residual gather: nodes per tile, wavefronts per node set
// node tiles of the multigrid sweeps: long in x, so that a wavefront reads every operator stream
// in runs of 256-512 contiguous bytes
constexpr int MGT2X = 64, MGT2Y = 4;
constexpr int MGT3X = 64, MGT3Y = 2, MGT3Z = 2;

// Particle state, structure of arrays: field f, component c of particle i lives at
// base[(f + c) * stride + i].  Every variant uses the same slots (2D leaves some unused).
enum PField : int {
    PX = 0,      // position (3)
    PF = 3,      // deformation gradient, row-major dim x dim (9)
    PV = 12,     // current volume V_n
    PM = 13,     // mass
    PP = 14,     // pore pressure
    PU = 15,     // accumulated displacement (3)
    PLP = 18,    // GIMP half-lengths (3)
    PLP0 = 21,   // initial GIMP half-lengths (3)
    PVEL = 24,   // velocity (3)
    PACC = 27,   // acceleration (3)
    PPD = 30,    // pdot
    PPDD = 31,   // pddot
    PSIG = 32,   // effective Cauchy stress xx yy zz xy yz xz (6)
    NPF = 38
};

// Error flags (device int array, one slot per meaning)
enum Flag : int { FL_INVERTED = 0, FL_OUTSIDE = 1, FL_NONFINITE = 2, FL_BOUNDS = 3, NFLAG = 4 };

// Scalars of one problem (device double array)
enum Scal : int {
    SC_RU2 = 0,      // ||R_u||^2
    SC_RP2 = 1,      // ||R_p||^2
    SC_RHO = 2,      // BiCGStab rho
    SC_ALPHA = 3,
    SC_OMEGA = 4,
    SC_BETA = 5,
    SC_RR = 6,       // ||r||^2
    SC_TOL2 = 7,     // (krylov tol * ||b||)^2
    SC_RV = 8,       // (rhat, v)
    SC_TS = 9,       // (t, s)
    SC_TT = 10,      // (t, t)
    SC_ITER = 11,    // iterations done (as double)
    SC_DONE = 12,    // 1 when converged or broken down
    SC_BREAK = 13,   // 1 on breakdown
    SC_MMAX = 14,    // largest nodal mass of the step (Stage 1)
    SC_BEST = 15,    // smallest ||r||^2 seen at a chunk end (its iterate is kept in kxb)
    SC_SREF = 16,    // ||r||^2 when the stagnation count last restarted
    SC_SITER = 17,   // iteration count at that restart
    SC_RESTART = 18, // 1: breakdown in k_bicg_s, rest of the iteration skipped; 2: the next
                     // iteration restarts from the current residual (rhat = p = r)
    SC_NRESTART = 19,// restarts of this solve
    NSCAL = 20
};

struct MgLevel {
    int n[3];            // nodes per axis
    int cz[3];           // 1 if the axis is coarsened towards the next level
    int np[3];           // padded nodes per axis
    int64_t nrow;        // prod n
    int64_t npad;        // prod np
    // operator of family A (block B = dim) and family S (block 1) on this level; level 0 uses
    // views into the Jacobian instead (null here)
    void* A;             // [S][dim][dim][nrow], T
    void* Ad;            // inverse diagonal blocks [dim*dim][nrow], T
    void* Sm;            // [S][nrow], T
    void* Sd;            // [nrow], T
    void* xa; void* ra; void* ba;   // family A: solution, residual, right-hand side [npad*dim]
    void* xs; void* rs; void* bsv;  // family S: solution, residual, right-hand side [npad]
};

// Device-side descriptor of one problem.  Lives in the problem's workspace; kernels of a batch
// receive pointers to the descriptors of all its problems.
struct Dev {
    int dim, shape, dyn, mixed, model;
    int R;        // stencil radius (= grid padding): 1 original MPM, 2 GIMP
    int W;        // basis nodes per axis and particle: 2 original MPM, 3 GIMP
    int S;        // stencil points (2R+1)^dim
    int b;        // dofs per node dim+1
    int nc[3];    // cells per axis
    int nn[3];    // real nodes per axis
    int np1[3];   // padded nodes per axis
    int64_t Np, Ncell, Nnode, Npad;
    double h, x0[3], hi[3];
    double lam, G, kappa, rho_f, g[3];
    double phi0;  // initial porosity of the Kozeny-Carman law, 0: constant mobility
    double alpha_vis;  // Kelvin-type damping parameter (dynamic problems)
    // per-step parameters
    double dt, beta, gamma, ct, tau, hc1, hc2, Kfs, omega;
    double kin;   // inertia factor of the Newmark fixed-stress modulus (fs_term)
    int schur;    // Schur-block form: 0 fixed-stress, 1 diagonal-inverse (lev[0].Sm holds it)
    int drain;    // 1: zero pore pressure on the free surface of the material (k_drain_surface)
    double negl;  // negligible-mass fraction (k_cut_light_nodes)
    // consistent-mass mapping of the P2G fields (kern_mass.hip), when cons is set
    int cons;
    int ncol;         // mapped fields: p (quasi-static); p, v, a, pdot, pddot (dynamic: 2 dim + 3)
    double* mrow;     // [S][Nnode] consistent mass rows over the fixed stencil (natural node order)
    double* mb;       // [ncol][Nnode] right-hand sides sum S m f
    double* mx;       // [ncol][Nnode] CG iterate (the mapped fields)
    double* mr;       // [ncol][Nnode] residual
    double* mz;       // [ncol][Nnode] preconditioned residual
    double* md;       // [ncol][Nnode] search direction
    double* mq;       // [ncol][Nnode] M d
    uint8_t* mheavy;  // [Nnode] 1: row solved with the consistent mass; 0: lumped value kept
    double* mpart;    // [maxblocks][3 MCOL] block partials
    double* mscal;    // [MCOL * 8 + 8] per-column CG scalars, then problem-wide slots
    int nlev;
    int ltail;    // first level handled by the fused small-level kernel
    int ls_stop;  // Schur-block hierarchy ends here with two Jacobi sweeps (>= ltail: not truncated)
    int mg_nsm;
    // particles
    double* pc;   // committed state
    double* pw;   // working copy of the step (sorted)
    int* idc;
    int* idw;
    int64_t ps;   // particle stride (= Np)
    // counting sort
    int* key;
    int* slot;
    int* ccount;  // [Ncell + 1]
    int* cstart;  // [Ncell + 1]
    int* order;   // [Np]
    // nodal fields on the padded grid
    double* M;
    double* Pn;
    double* vn;   // [Npad*3]
    double* an;   // [Npad*3]
    double* pdn;
    double* pddn;
    double* Mp;   // lumped pressure mass sum V_n S (fixed-stress Schur approximation)
    uint8_t* dfree;   // [Npad*b] 1 = free dof
    uint8_t* bcfix;   // [Npad*b]
    double* bcval;    // [Npad*b] u increment / p value
    double* fext;     // [Npad*b] f_ext, -q_ext
    double* X;        // [Npad*b] Newton iterate U, P
    double* Rv;       // [Npad*b] residual
    double* cellpi;   // [Ncell * 2^dim] original-MPM projection Pi N
    // quadrature-point records
    double* rec;      // point records, NREC contiguous words per point (RecRef)
    // Jacobian, fixed stencil block rows: entry e = (s*b + a)*b + c of row r at
    // J[jidx<dim>(e, r, S*b*b, Nnode)], precision T (see jidx)
    void* J;
    // 3D: cell matrices [Ncell][16][64] (entry, node pair), precision T
    void* Ke;
    // Krylov vectors [Npad*b], precision T
    void* kx; void* kr; void* kh; void* kp; void* kv; void* ks; void* kt; void* kph; void* ksh;
    void* kxb;        // [Npad*b] iterate of the smallest residual seen at a chunk end
    void* kbt;        // [Npad*dim] rhs of the A cycle (r_u - B1 z_p)
    // multigrid hierarchy
    MgLevel lev[MAXLEV];
    void* cinvA;      // dense inverse of the coarsest A [nA*nA], precision T
    void* cinvS;      // dense inverse of the coarsest S [nS*nS], precision T
    double* cwork;    // FP64 Gauss-Jordan work matrix [CMAX*CMAX]
    // reductions
    double* partial;  // [maxblocks * 4]
    double* scal;     // [NSCAL]
    int* flags;       // [NFLAG]
    int64_t maxblocks;
};

// Jacobian storage.  3D: rows in blocks of JB, entry-major inside a block, so that a wavefront's
// whole block row (432 words per row) is one contiguous run.  2D: entry-major over all rows,
// J[e * Nnode + row] (the 2D Jacobian is small enough to stay largely in the 256 MB Infinity
// Cache, and this order measured faster there).  Both give 64 consecutive words per entry for a
// wavefront of 64 consecutive rows.
constexpr int JB = 64;
template <int DIM>
__host__ __device__ __forceinline__ int64_t jidx(int e, int64_t row, int NE, int64_t nrow) {
    if (DIM == 3) return (row >> 6) * ((int64_t)NE << 6) + ((int64_t)e << 6) + (row & 63);
    return (int64_t)e * nrow + row;
}
__host__ __device__ __forceinline__ int64_t jrows_padded(int64_t nrow) { return (nrow + JB - 1) / JB * JB; }

// SpMV launch shape, the number of blocks (and of reduction partials) of a problem.  FP64: one
// wavefront per (component row a, run of 64 consecutive nodes), four wavefronts per block;
// FP32: one thread per node.
__host__ __device__ __forceinline__ int64_t spmv_blocks(int dim, int64_t nnode, bool fp64) {
    if (!fp64) return (nnode + TPB - 1) / TPB;
    const int64_t waves = (nnode + 63) / 64 * (dim + 1);
    return (waves + 3) / 4;
}

// Batch of problems of one kernel variant, passed by value to every kernel.
struct Batch {
    int n;
    int pfx[MAXB + 1];         // block prefix: problem q owns blocks [pfx[q], pfx[q+1])
    const Dev* d[MAXB];
};

__device__ __forceinline__ int batch_find(const Batch& B, int blk) {
    // problems are few: linear scan on uniform data
    int q = 0;
    while (q + 1 < B.n && blk >= B.pfx[q + 1]) ++q;
    return q;
}

// ------------------------------------------------------------------------------------------------
// record layout (quadrature-point data written once per Newton iteration): the fields the
// residual gather reads come first, so that one visit touches three cache lines instead of four
// ------------------------------------------------------------------------------------------------
template <int DIM, int WB>
struct RecLayout {
    static constexpr int W_ = 0;                      // 1D weights [DIM][WB]
    static constexpr int DW_ = W_ + DIM * WB;          // 1D gradients [DIM][WB]
    static constexpr int S0_ = DW_ + DIM * WB;         // GIMP constant basis [DIM][WB]
    static constexpr int FI_ = S0_ + DIM * WB;         // dF^{-1} [DIM*DIM]
    static constexpr int SG_ = FI_ + DIM * DIM;        // -V0 tau' + dv p 1 [DIM*DIM]
    static constexpr int BF_ = SG_ + DIM * DIM;        // m (g - a) [DIM]
    static constexpr int DT_ = BF_ + DIM;              // dv theta
    static constexpr int ST_ = DT_ + 1;                // tau V_n (pdot - Pi pdot)
    static constexpr int DK_ = ST_ + 1;                // dv kappa
    static constexpr int QW_ = DK_ + 1;                // w = grad p - rho_f (g - a) [DIM]
    static constexpr int AB_ = QW_ + DIM;              // tangent Abar [DIM^4]
    static constexpr int DV_ = AB_ + DIM * DIM * DIM * DIM;   // dv
    static constexpr int CM_ = DV_ + 1;                // m / (beta dt^2)
    static constexpr int BV_ = CM_ + 1;                // volumetric coupling coefficient
    static constexpr int LV_ = BV_ + 1;                // dv * velocity gradient [DIM*DIM]
    static constexpr int GP_ = LV_ + DIM * DIM;        // grad p [DIM]
    static constexpr int EE_ = GP_ + DIM;              // dv kappa rho_f / (beta dt^2)
    static constexpr int TC_ = EE_ + 1;                // tau c_t V_n
    static constexpr int KJ_ = TC_ + 1;                // dv J dkappa/dJ (Kozeny-Carman; else 0)
    static constexpr int N = KJ_ + 1;
};

// 3D (trilinear, neo-Hookean): no folded tangent.  The cell-matrix kernel forms the
// displacement block of each node pair in closed form from V0 G, b = F F^T and two scalars:
//   A_ik^ac = -V0 G (gi . b gk) d_ac + C1 gk_a gi_c + C2 gi_a gk_c
//   C1 = V0 (lam ln J - G) - dv p,   C2 = dv p - V0 lam
// (plus the Newmark inertia and the Kelvin damping terms), which is the contraction
// gi_b Abar_{ab,ce} gk_e of the folded tangent for tau' = G (b - 1) + lam ln J 1.
// 80 words = five 128-byte lines: every record starts on a line, the residual gather's 39 words
// are its first three lines and the cell-matrix kernel's 66 words its first five.
template <>
struct RecLayout<3, 2> {
    static constexpr int W_ = 0;       // 1D weights [3][2]
    static constexpr int DW_ = 6;      // 1D gradients [3][2]
    static constexpr int FI_ = 12;     // dF^{-1} [9]
    static constexpr int SG_ = 21;     // -V0 tau' + dv p 1 - dv sigma_vis [9]
    static constexpr int BF_ = 30;     // m (g - a) [3]
    static constexpr int DT_ = 33;     // dv theta
    static constexpr int ST_ = 34;     // tau V_n (pdot - Pi pdot)
    static constexpr int DK_ = 35;     // dv kappa
    static constexpr int QW_ = 36;     // w = grad p - rho_f (g - a) [3]
    static constexpr int DV_ = 39;     // dv
    static constexpr int CM_ = 40;     // m / (beta dt^2)
    static constexpr int BV_ = 41;     // volumetric coupling coefficient
    static constexpr int LV_ = 42;     // dv * velocity gradient [9]
    static constexpr int GP_ = 51;     // grad p [3]
    static constexpr int EE_ = 54;     // dv kappa rho_f / (beta dt^2)
    static constexpr int TC_ = 55;     // tau c_t V_n
    static constexpr int KJ_ = 56;     // dv J dkappa/dJ (Kozeny-Carman; else 0)
    static constexpr int VG_ = 57;     // V0 G
    static constexpr int BM_ = 58;     // b = F F^T: xx yy zz xy yz xz
    static constexpr int C1_ = 64;
    static constexpr int C2_ = 65;
    static constexpr int SV_ = 66;     // sigma_vis: xx yy zz xy yz xz (Kelvin damping only)
    static constexpr int S0_ = 72;     // (GIMP constant basis; unused by the trilinear basis) [3][2]
    static constexpr int N = 80;
};

// Record of point p: NREC contiguous words (the gathers read ~30 fields of one point per visit,
// which then share a few cache lines).  rec[f] is field f of the point.
struct RecRef {
    double* b;
    __device__ __forceinline__ RecRef(double* base, int64_t p, int nrec) : b(base + p * nrec) {}
    __device__ __forceinline__ double& operator[](int f) const { return b[f]; }
};
__host__ __device__ __forceinline__ int64_t rec_points_padded(int64_t np) { return np; }

// Kozeny-Carman mobility (Sec. 2.2, eq. kozeny-carman) at volume ratio J for initial porosity
// phi0 > 0: with phi = 1 - (1 - phi0)/J (incompressible grains), kappa = kappa0 (phi/phi0)^3
// ((1 - phi0)/(1 - phi))^2.  Also *kj = J dkappa/dJ = kappa (3 - phi)/phi, the extra factor of the
// mass-balance linearization; below KC_PHI_MIN the porosity is held there and *kj = 0.
constexpr double KC_PHI_MIN = 1e-4;
__device__ __forceinline__ void kozeny_carman(double kappa0, double phi0, double J, double* k, double* kj) {
    double phi = 1.0 - (1.0 - phi0) / J;
    const bool held = !(phi >= KC_PHI_MIN);
    if (held) phi = KC_PHI_MIN;
    const double r = phi / phi0, q = (1.0 - phi0) / (1.0 - phi);
    *k = kappa0 * r * r * r * q * q;
    *kj = held ? 0.0 : *k * (3.0 - phi) / phi;
}

// ------------------------------------------------------------------------------------------------
// basis functions (Sec. 3.1)
// ------------------------------------------------------------------------------------------------

// Antiderivative of the unit hat of half-width h, int_{-inf}^{r} N: clamp-based form.
__device__ __forceinline__ double hat_prim(double r, double h) {
    double c = fmin(fmax(r, -h), h);
    return 0.5 * h + c - c * fabs(c) / (2.0 * h);
}
__device__ __forceinline__ double hat_val(double r, double h) { return fmax(0.0, 1.0 - fabs(r) / h); }

// First node of a particle's basis window along one axis (its sort bucket, too): original MPM
// the cell containing x; GIMP the node at or left of the lower end of the domain [x-lp, x+lp]
// clipped to the grid; clamped to the cells.  Sort keys and the basis use this one function, so
// the bucket of a particle is exactly its window base.
template <int SHAPE>
__device__ __forceinline__ int window_base(double x, double lp, double x0, double h, int nc) {
    const double a = SHAPE == 0 ? x : fmax(x - lp, x0);
    int c = (int)floor((a - x0) / h);
    return c < 0 ? 0 : (c > nc - 1 ? nc - 1 : c);
}

// Overlap (relative to h) below which a GIMP domain and a node's support only touch: the
// intersection has measure zero and the node gets weight, gradient and S0 exactly 0, so that the
// rounding of the interval ends cannot make an untouched node active with a ~1e-27 mass.
constexpr double GIMP_TOUCH = 1e-10;

// A node whose mass is below this fraction of the step's largest nodal mass (a point domain that
// only just reaches its support) is outside the material: its rows would be ~1e-18 of the others
// and the Newton update there unbounded.
constexpr double NEGLIGIBLE_MASS = 1e-15;   // default of ppmpm_options.negligible_mass

// 1D basis of one particle along one axis.  Original MPM: the two nodes of the containing cell
// (clamped), hat weights.  GIMP: the domain [x-lp, x+lp] clipped to the grid, three nodes from
// the one at or left of its lower end; weight = domain average of the hat, gradient = domain
// average of its derivative (= (N(b) - N(a)) / |[a,b]|), constant basis S0 = half the share of
// the domain inside the node's support.
template <int SHAPE>
__device__ __forceinline__ int basis_1d(double x, double lp, double x0, double h, int nc, double* w,
                                        double* dw, double* s0) {
    const int base = window_base<SHAPE>(x, lp, x0, h, nc);
    if (SHAPE == 0) {
        double xi = (x - (x0 + h * base)) / h;
        w[0] = 1.0 - xi;
        w[1] = xi;
        dw[0] = -1.0 / h;
        dw[1] = 1.0 / h;
        s0[0] = s0[1] = 0.5;
    } else {
        double lo = x0, hi = x0 + h * nc;
        double a = fmax(x - lp, lo), bb = fmin(x + lp, hi);
        double len = bb - a;
        for (int k = 0; k < 3; ++k) {
            double xn = x0 + h * (base + k);
            w[k] = (hat_prim(bb - xn, h) - hat_prim(a - xn, h)) / len;
            dw[k] = (hat_val(bb - xn, h) - hat_val(a - xn, h)) / len;
            double ov = fmin(bb, xn + h) - fmax(a, xn - h);
            const bool in = ov > GIMP_TOUCH * h;
            s0[k] = in ? 0.5 * ov / len : 0.0;
            if (!in) w[k] = dw[k] = 0.0;
        }
    }
    return base;
}

// ------------------------------------------------------------------------------------------------
// small dense helpers
// ------------------------------------------------------------------------------------------------
template <int D>
__device__ __forceinline__ double det(const double* A) {
    if (D == 2) return A[0] * A[3] - A[1] * A[2];
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

template <int D>
__device__ __forceinline__ void inverse(const double* A, double* B) {
    double id = 1.0 / det<D>(A);
    if (D == 2) {
        B[0] = A[3] * id; B[1] = -A[1] * id; B[2] = -A[2] * id; B[3] = A[0] * id;
    } else {
        B[0] = (A[4] * A[8] - A[5] * A[7]) * id;
        B[1] = (A[2] * A[7] - A[1] * A[8]) * id;
        B[2] = (A[1] * A[5] - A[2] * A[4]) * id;
        B[3] = (A[5] * A[6] - A[3] * A[8]) * id;
        B[4] = (A[0] * A[8] - A[2] * A[6]) * id;
        B[5] = (A[2] * A[3] - A[0] * A[5]) * id;
        B[6] = (A[3] * A[7] - A[4] * A[6]) * id;
        B[7] = (A[1] * A[6] - A[0] * A[7]) * id;
        B[8] = (A[0] * A[4] - A[1] * A[3]) * id;
    }
}

// (ln x - ln y)/(x - y) for positive x, y, continuous across x = y.
__device__ __forceinline__ double log_divdiff(double x, double y) {
    double t = (x - y) / y;
    if (fabs(t) < 1e-4) {
        // log1p(t)/t = 1 - t/2 + t^2/3 - t^3/4 + t^4/5
        return (1.0 + t * (-0.5 + t * (1.0 / 3.0 + t * (-0.25 + t * 0.2)))) / y;
    }
    return log1p(t) / (x - y);
}

// Effective Kirchhoff stress tau' (full DIM x DIM block, plus tau'_zz in plane strain) and the
// tangent T with d tau' = T : L for dF -> (1 + L) dF (L = d(grad u) in the current configuration):
//   neo-Hookean: tau' = G (b - 1) + lam ln J 1,   T_abef = G (d_ae b_fb + b_af d_be) + lam d_ab d_ef
//   Hencky:      tau' = lam ln J 1 + G ln b,      T = lam 1(x)1 + G D(ln b)[L b + b L^T]
// (the Hencky derivative by the Daleckii-Krein formula in the eigenframe of b; plane strain only).
template <int D>
__device__ __forceinline__ void kirchhoff_tangent(int model, double lam, double G, const double* F,
                                                  double* tau, double* tauzz, double* T) {
    double b[9];
    for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) {
            double s = 0.0;
            for (int k = 0; k < D; ++k) s += F[i * D + k] * F[j * D + k];
            b[i * D + j] = s;
        }
    double lnJ = log(det<D>(F));
    if (model == 1 || D == 3) {
        for (int i = 0; i < D * D; ++i) tau[i] = G * b[i];
        for (int i = 0; i < D; ++i) tau[i * D + i] += lam * lnJ - G;
        *tauzz = lam * lnJ;
        if (T) {
            for (int a = 0; a < D; ++a)
                for (int bb = 0; bb < D; ++bb)
                    for (int e = 0; e < D; ++e)
                        for (int f = 0; f < D; ++f) {
                            double v = 0.0;
                            if (a == e) v += G * b[f * D + bb];
                            if (bb == e) v += G * b[a * D + f];
                            if (a == bb && e == f) v += lam;
                            T[((a * D + bb) * D + e) * D + f] = v;
                        }
        }
        return;
    }
    // Hencky, 2x2: principal frame of b by the half angle
    double th = 0.5 * atan2(2.0 * b[1], b[0] - b[3]);
    double cs = cos(th), sn = sin(th);
    double Q[4] = {cs, -sn, sn, cs};   // columns: n1 = (cs, sn), n2 = (-sn, cs)
    double l1 = b[0] * cs * cs + 2.0 * b[1] * cs * sn + b[3] * sn * sn;
    double l2 = b[0] * sn * sn - 2.0 * b[1] * cs * sn + b[3] * cs * cs;
    double e1 = log(l1), e2 = log(l2);
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            tau[i * 2 + j] = G * (Q[i * 2] * e1 * Q[j * 2] + Q[i * 2 + 1] * e2 * Q[j * 2 + 1]) +
                             (i == j ? lam * lnJ : 0.0);
    *tauzz = lam * lnJ;
    if (!T) return;
    double ev[2] = {l1, l2};
    double gdd[4];
    gdd[0] = 1.0 / l1;
    gdd[3] = 1.0 / l2;
    gdd[1] = gdd[2] = log_divdiff(l1, l2);
    // eigenframe tangent T'_ABEF = lam d_AB d_EF + G g_AB (l_B d_AE d_BF + l_A d_BE d_AF)
    double Tp[16];
    for (int A = 0; A < 2; ++A)
        for (int Bq = 0; Bq < 2; ++Bq)
            for (int E = 0; E < 2; ++E)
                for (int Fq = 0; Fq < 2; ++Fq) {
                    double v = (A == Bq && E == Fq) ? lam : 0.0;
                    double gg = gdd[A * 2 + Bq];
                    if (A == E && Bq == Fq) v += G * gg * ev[Bq];
                    if (Bq == E && A == Fq) v += G * gg * ev[A];
                    Tp[((A * 2 + Bq) * 2 + E) * 2 + Fq] = v;
                }
    for (int a = 0; a < 2; ++a)
        for (int bb = 0; bb < 2; ++bb)
            for (int e = 0; e < 2; ++e)
                for (int f = 0; f < 2; ++f) {
                    double v = 0.0;
                    for (int A = 0; A < 2; ++A)
                        for (int Bq = 0; Bq < 2; ++Bq) {
                            double qab = Q[a * 2 + A] * Q[bb * 2 + Bq];
                            for (int E = 0; E < 2; ++E)
                                for (int Fq = 0; Fq < 2; ++Fq)
                                    v += qab * Q[e * 2 + E] * Q[f * 2 + Fq] * Tp[((A * 2 + Bq) * 2 + E) * 2 + Fq];
                        }
                    T[((a * 2 + bb) * 2 + e) * 2 + f] = v;
                }
}

// padded node index of a real node
__device__ __forceinline__ int64_t pad_index(const Dev* d, int ix, int iy, int iz) {
    int R = d->R;
    if (d->dim == 2) return (int64_t)(ix + R) + (int64_t)d->np1[0] * (iy + R);
    return (int64_t)(ix + R) + (int64_t)d->np1[0] * ((iy + R) + (int64_t)d->np1[1] * (iz + R));
}

// *addr = max(*addr, max over the block's m) for non-negative m (their bit patterns order like
// the values): a shuffle tree per wavefront, then one atomic per block that holds a positive m.
// Every thread of the block must call it (it has a barrier).
__device__ __forceinline__ void block_max_nonneg(double* addr, double m) {
    __shared__ double wmax[TPB / 64];
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = wmax[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) b = fmax(b, wmax[w]);
        if (b > 0.0) atomicMax((unsigned long long*)addr, (unsigned long long)__double_as_longlong(b));
    }
}

}  // namespace ppm
