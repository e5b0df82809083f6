/*
 * oracle.c -- plain, slow, single-threaded FP64 reference of the stabilized implicit MPM for
 * coupled large-deformation poromechanics of Zhao & Choo (arXiv 1905.00671).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or calls this
 * file; only the test-suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 * It shares no code, header, table or constant with the HIP library.
 *
 * Conventions
 *   dim = 2 (plane strain, F_zz = 1) or 3.  Nodes of the fixed background grid are numbered
 *   ix + nx1*(iy + ny1*iz).  Nodal unknowns are the incremental displacement U (dim) and the
 *   pore pressure P; degree of freedom (node, c) = node*(dim+1) + c, c = dim is the pressure.
 *   Particle arrays are flat, row-major ([np*dim], [np*dim*dim], ...).
 *
 * Every routine follows the passage of the paper named in its comment; where the paper is
 * silent the reading used is named the same way (readings are listed with the design notes).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXN 64 /* nodes per particle: GIMP 3D 4^3 */

typedef struct {
    int dim;
    int nc[3];
    double h;
    double x0[3];
} or_grid;

typedef struct {
    int model;       /* 0 Hencky (Sec. 2.2), 1 neo-Hookean */
    double lam, G;   /* Lame parameters */
    double kappa;    /* mobility k / mu_f (Darcy law, Sec. 2.2) */
    double rho_f;
    double g[3];
    double phi0;     /* initial porosity of the Kozeny-Carman law (Sec. 2.2); <= 0: kappa constant */
    double alpha_vis; /* damping parameter of the Kelvin-type viscous stress (Sec. 2.2); dynamic only */
} or_mat;

/* Porosity below which the Kozeny-Carman mobility is held constant (the law degenerates at
 * phi = 0, where the grains alone would fill the volume). */
#define OR_PHI_MIN 1e-4

typedef struct {
    int shape;       /* 0 original MPM, 1 GIMP */
    int dynamic;     /* 0 quasi-static implicit Euler, 1 Newmark */
    double beta, gamma, dt;
    double tau;      /* PPP stabilization parameter (0: off) */
} or_opt;

/* ------------------------------------------------------------------------------------------ */
/* small dense helpers                                                                         */
/* ------------------------------------------------------------------------------------------ */

static double det_n(int d, const double* A) {
    if (d == 2) return A[0] * A[3] - A[1] * A[2];
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

static void inv_n(int d, const double* A, double* B) {
    double D = det_n(d, A);
    if (d == 2) {
        B[0] = A[3] / D; B[1] = -A[1] / D; B[2] = -A[2] / D; B[3] = A[0] / D;
        return;
    }
    B[0] = (A[4] * A[8] - A[5] * A[7]) / D;
    B[1] = (A[2] * A[7] - A[1] * A[8]) / D;
    B[2] = (A[1] * A[5] - A[2] * A[4]) / D;
    B[3] = (A[5] * A[6] - A[3] * A[8]) / D;
    B[4] = (A[0] * A[8] - A[2] * A[6]) / D;
    B[5] = (A[2] * A[3] - A[0] * A[5]) / D;
    B[6] = (A[3] * A[7] - A[4] * A[6]) / D;
    B[7] = (A[1] * A[6] - A[0] * A[7]) / D;
    B[8] = (A[0] * A[4] - A[1] * A[3]) / D;
}

static void matmul_n(int d, const double* A, const double* B, double* C) {
    for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++) {
            double s = 0.0;
            for (int k = 0; k < d; k++) s += A[i * d + k] * B[k * d + j];
            C[i * d + j] = s;
        }
}

/* ------------------------------------------------------------------------------------------ */
/* basis functions (Sec. 3.1)                                                                  */
/* ------------------------------------------------------------------------------------------ */

/* Linear hat of half-width h centred at 0. */
static double hat(double r, double h) {
    double a = fabs(r);
    return a < h ? 1.0 - a / h : 0.0;
}

/* Antiderivative of the hat: int_{-inf}^{r} hat(s) ds, written piece by piece. */
static double hat_int(double r, double h) {
    if (r <= -h) return 0.0;
    if (r <= 0.0) return (r + h) * (r + h) / (2.0 * h);
    if (r <= h) return h - (h - r) * (h - r) / (2.0 * h);
    return h;
}

/* 1D GIMP weight and gradient of the node at xi for a particle domain [a, b] (eq. gimp-basis
 * and gimp-basis-gradient): S = (1/|[a,b]|) int_a^b N dxi, dS = (1/|[a,b]|) int_a^b N' dxi.
 * The domain has already been intersected with the grid (the "cap Omega" of the definition);
 * dividing by the clipped length keeps the partition of unity (reading for domains touching
 * the grid boundary). */
static void gimp_1d(double a, double b, double xi, double h, double* S, double* dS) {
    double len = b - a;
    *S = (hat_int(b - xi, h) - hat_int(a - xi, h)) / len;
    *dS = (hat(b - xi, h) - hat(a - xi, h)) / len;
}

/* Overlap (relative to h) below which a node's support and a particle domain only touch: the
 * intersection of the definition (eq. gimp-basis) then has measure zero and the node carries no
 * weight.  Without the threshold, the rounding of the interval ends (cell sizes that are not
 * powers of two) would decide whether such a node gets a mass of ~1e-27 and becomes active. */
#define OR_GIMP_TOUCH 1e-10

/* 1D constant basis of the GIMP-compatible projection (Sec. 4.4): one half of the share of the
 * particle domain lying inside the support [xi - h, xi + h] of the node; 0 (and the node is not
 * in the point's basis) when the two only touch. */
static double gimp_s0_1d(double a, double b, double xi, double h) {
    double lo = a > xi - h ? a : xi - h;
    double hi = b < xi + h ? b : xi + h;
    double ov = hi - lo;
    return ov > OR_GIMP_TOUCH * h ? 0.5 * ov / (b - a) : 0.0;
}

static int cell_of(const or_grid* g, int d, double x) {
    int c = (int)floor((x - g->x0[d]) / g->h);
    if (c < 0) c = 0;
    if (c > g->nc[d] - 1) c = g->nc[d] - 1;
    return c;
}

/* Basis of one material point: list of nodes with their weight S, reference gradient G = grad_n S
 * (gradient with respect to the configuration at t_n, where the basis is evaluated through the
 * whole step, Sec. 3.3) and, for GIMP, the constant projection basis S0.
 * Original MPM: the 2^dim nodes of the containing cell, FE hat product.  GIMP: every node whose
 * support overlaps the particle domain.  Returns the number of nodes. */
int or_basis(const or_grid* g, int shape, const double* xp, const double* lp, int* nodes, double* S,
             double* G, double* S0) {
    int d = g->dim;
    int n1[3] = {g->nc[0] + 1, g->nc[1] + 1, d == 3 ? g->nc[2] + 1 : 1};
    int cnt[3] = {1, 1, 1}, base[3] = {0, 0, 0};
    double w[3][4], dw[3][4], w0[3][4];
    for (int a = 0; a < d; a++) {
        int c = cell_of(g, a, xp[a]);
        if (shape == 0) {
            base[a] = c;
            cnt[a] = 2;
            double xl = g->x0[a] + g->h * c;
            for (int k = 0; k < 2; k++) {
                double xi = xl + g->h * k;
                double r = xp[a] - xi;
                w[a][k] = 1.0 - fabs(r) / g->h;
                if (w[a][k] < 0.0) w[a][k] = 0.0;
                dw[a][k] = (k == 0) ? -1.0 / g->h : 1.0 / g->h;
                w0[a][k] = 0.5;
            }
        } else {
            double lo = g->x0[a], hi = g->x0[a] + g->h * g->nc[a];
            double A = xp[a] - lp[a], B = xp[a] + lp[a];
            if (A < lo) A = lo;
            if (B > hi) B = hi;
            base[a] = c - 1;
            cnt[a] = 4;
            for (int k = 0; k < 4; k++) {
                int ni = c - 1 + k;
                double xi = g->x0[a] + g->h * ni;
                if (ni < 0 || ni > g->nc[a]) {
                    w[a][k] = dw[a][k] = w0[a][k] = 0.0;
                    continue;
                }
                gimp_1d(A, B, xi, g->h, &w[a][k], &dw[a][k]);
                w0[a][k] = gimp_s0_1d(A, B, xi, g->h);
            }
        }
    }
    int n = 0;
    for (int k2 = 0; k2 < cnt[2]; k2++)
        for (int k1 = 0; k1 < cnt[1]; k1++)
            for (int k0 = 0; k0 < cnt[0]; k0++) {
                int kk[3] = {k0, k1, k2};
                int idx[3];
                int skip = 0;
                for (int a = 0; a < d; a++) {
                    idx[a] = base[a] + kk[a];
                    if (idx[a] < 0 || idx[a] >= n1[a]) skip = 1;
                    if (shape == 1 && w0[a][kk[a]] == 0.0) skip = 1; /* no overlap */
                }
                if (skip) continue;
                double s = 1.0, s0 = 1.0;
                for (int a = 0; a < d; a++) {
                    s *= w[a][kk[a]];
                    s0 *= w0[a][kk[a]];
                }
                for (int a = 0; a < d; a++) {
                    double gr = 1.0;
                    for (int b = 0; b < d; b++) gr *= (b == a) ? dw[b][kk[b]] : w[b][kk[b]];
                    G[n * d + a] = gr;
                }
                nodes[n] = idx[0] + n1[0] * (idx[1] + n1[1] * (d == 3 ? idx[2] : 0));
                S[n] = s;
                if (S0) S0[n] = s0;
                n++;
            }
    return n;
}

/* ------------------------------------------------------------------------------------------ */
/* constitutive laws (Sec. 2.2)                                                                */
/* ------------------------------------------------------------------------------------------ */

/* Eigen-decomposition of a symmetric 2x2 matrix by one Jacobi rotation. */
static void eig_sym2(const double* A, double* lam, double* Q) {
    double a = A[0], c = A[1], d = A[3];
    if (c == 0.0) {
        lam[0] = a; lam[1] = d;
        Q[0] = 1; Q[1] = 0; Q[2] = 0; Q[3] = 1;
        return;
    }
    double th = (d - a) / (2.0 * c);
    double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
    double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
    lam[0] = a - t * c;
    lam[1] = d + t * c;
    /* columns are the eigenvectors: v0 = (cs, -sn), v1 = (sn, cs) */
    Q[0] = cs; Q[1] = sn; Q[2] = -sn; Q[3] = cs;
}

/* (ln x - ln y)/(x - y), continuous at x = y. */
static double dlog_dd(double x, double y) {
    double r = x / y - 1.0;
    if (fabs(r) < 1e-5) return (1.0 - r / 2.0 + r * r / 3.0 - r * r * r / 4.0) / y;
    return log1p(r) / (x - y);
}

/* Effective Kirchhoff stress tau' = J sigma' as a full 3x3 tensor from the deformation
 * gradient F (dim x dim; plane strain has F_zz = 1).
 *   Hencky (the paper's model): Psi = lam/2 (ln J)^2 + G tr((1/2 ln b)^2)
 *                               => tau' = lam ln J 1 + G ln b.
 *   Neo-Hookean reading:        tau' = G (b - 1) + lam ln J 1. */
void or_kirchhoff(int model, double lam, double G, int d, const double* F, double* tau) {
    double b[9] = {0}, J = det_n(d, F);
    for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++) {
            double s = 0;
            for (int k = 0; k < d; k++) s += F[i * d + k] * F[j * d + k];
            b[i * 3 + j] = s;
        }
    if (d == 2) b[8] = 1.0;
    double lnJ = log(J);
    memset(tau, 0, 9 * sizeof(double));
    if (model == 1) {
        for (int i = 0; i < 9; i++) tau[i] = G * b[i];
        for (int i = 0; i < 3; i++) tau[i * 4] += -G + lam * lnJ;
        return;
    }
    /* Hencky: only plane strain is supported by this reference */
    double b2[4] = {b[0], b[1], b[3], b[4]}, ev[2], Q[4];
    eig_sym2(b2, ev, Q);
    double l0 = log(ev[0]), l1 = log(ev[1]);
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++)
            tau[i * 3 + j] = G * (Q[i * 2 + 0] * l0 * Q[j * 2 + 0] + Q[i * 2 + 1] * l1 * Q[j * 2 + 1]);
    for (int i = 0; i < 3; i++) tau[i * 4] += lam * lnJ;
}

/* Directional derivative of tau' along the velocity-gradient-like direction L (dim x dim):
 * F -> F + eps L F, so that delta b = L b + b L^T and delta ln J = tr L. */
void or_dkirchhoff(int model, double lam, double G, int d, const double* F, const double* L,
                   double* dtau) {
    double b[9] = {0};
    for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++) {
            double s = 0;
            for (int k = 0; k < d; k++) s += F[i * d + k] * F[j * d + k];
            b[i * 3 + j] = s;
        }
    if (d == 2) b[8] = 1.0;
    double trL = 0;
    for (int i = 0; i < d; i++) trL += L[i * d + i];
    double db[9] = {0};
    for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++) {
            double s = 0;
            for (int k = 0; k < d; k++) s += L[i * d + k] * b[k * 3 + j] + b[i * 3 + k] * L[j * d + k];
            db[i * 3 + j] = s;
        }
    memset(dtau, 0, 9 * sizeof(double));
    if (model == 1) {
        for (int i = 0; i < 9; i++) dtau[i] = G * db[i];
        for (int i = 0; i < 3; i++) dtau[i * 4] += lam * trL;
        return;
    }
    /* Hencky: G * D(ln b)[db] by the Daleckii-Krein formula in the eigenbasis of b */
    double b2[4] = {b[0], b[1], b[3], b[4]}, ev[2], Q[4];
    eig_sym2(b2, ev, Q);
    double dbe[4] = {0}; /* Q^T db Q */
    for (int A = 0; A < 2; A++)
        for (int B = 0; B < 2; B++) {
            double s = 0;
            for (int i = 0; i < 2; i++)
                for (int j = 0; j < 2; j++) s += Q[i * 2 + A] * db[i * 3 + j] * Q[j * 2 + B];
            dbe[A * 2 + B] = s;
        }
    double gdd[4];
    gdd[0] = 1.0 / ev[0];
    gdd[3] = 1.0 / ev[1];
    gdd[1] = gdd[2] = dlog_dd(ev[0], ev[1]);
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) {
            double s = 0;
            for (int A = 0; A < 2; A++)
                for (int B = 0; B < 2; B++) s += Q[i * 2 + A] * gdd[A * 2 + B] * dbe[A * 2 + B] * Q[j * 2 + B];
            dtau[i * 3 + j] = G * s;
        }
    for (int i = 0; i < 3; i++) dtau[i * 4] += lam * trL;
}

/* ------------------------------------------------------------------------------------------ */
/* Stage 1: particles -> nodes (eq. map-from-particles-to-nodes)                               */
/* ------------------------------------------------------------------------------------------ */

/* Accumulates the lumped nodal sums M_i = sum S m and sum S m f for f in {p, v, a, pdot, pddot};
 * the caller divides by M_i.  Any of the output arrays except M may be NULL. */
void or_p2g(const or_grid* g, int shape, long np, const double* x, const double* lp, const double* m,
            const double* p, const double* v, const double* a, const double* pd, const double* pdd,
            double* M, double* Mp, double* Mv, double* Ma, double* Mpd, double* Mpdd) {
    int d = g->dim;
    int nodes[OR_MAXN];
    double S[OR_MAXN], G[OR_MAXN * 3];
    for (long q = 0; q < np; q++) {
        int n = or_basis(g, shape, x + q * d, lp ? lp + q * d : NULL, nodes, S, G, NULL);
        for (int k = 0; k < n; k++) {
            double w = S[k] * m[q];
            int i = nodes[k];
            M[i] += w;
            if (Mp) Mp[i] += w * p[q];
            if (Mpd) Mpd[i] += w * pd[q];
            if (Mpdd) Mpdd[i] += w * pdd[q];
            for (int c = 0; c < d; c++) {
                if (Mv) Mv[i * d + c] += w * v[q * d + c];
                if (Ma) Ma[i * d + c] += w * a[q * d + c];
            }
        }
    }
}

/* Consistent mass matrix of eq. map-from-particles-to-nodes-consistent, M_ij = sum_mp S_i S_j m,
 * as COO triplets: one per material point and ordered pair of its basis nodes (the caller sums
 * duplicates).  Capacity: np * OR_MAXN^2 triplets.  Returns the number written. */
long or_mass_matrix(const or_grid* g, int shape, long np, const double* x, const double* lp, const double* m,
                    long* ri, long* ci, double* v) {
    int d = g->dim;
    int nodes[OR_MAXN];
    double S[OR_MAXN], G[OR_MAXN * 3];
    long cnt = 0;
    for (long q = 0; q < np; q++) {
        int n = or_basis(g, shape, x + q * d, lp ? lp + q * d : NULL, nodes, S, G, NULL);
        for (int i = 0; i < n; i++)
            for (int j = 0; j < n; j++) {
                ri[cnt] = nodes[i];
                ci[cnt] = nodes[j];
                v[cnt] = S[i] * S[j] * m[q];
                cnt++;
            }
    }
    return cnt;
}

/* 1D weights of the nodes base..base+cnt-1 along axis a for a point at xa with half-length lpa:
 * the hat of the containing cell (original MPM) or the GIMP weights of eq. gimp-basis (domain
 * clipped to the grid, nodes whose support only touches the domain carry 0).  Returns cnt. */
static int axis_weights(const or_grid* g, int shape, int a, double xa, double lpa, int* base, double* w) {
    int c = cell_of(g, a, xa);
    if (shape == 0) {
        *base = c;
        double xl = g->x0[a] + g->h * c;
        for (int k = 0; k < 2; k++) {
            w[k] = 1.0 - fabs(xa - (xl + g->h * k)) / g->h;
            if (w[k] < 0.0) w[k] = 0.0;
        }
        return 2;
    }
    double lo = g->x0[a], hi = g->x0[a] + g->h * g->nc[a];
    double A = xa - lpa, B = xa + lpa;
    if (A < lo) A = lo;
    if (B > hi) B = hi;
    *base = c - 1;
    for (int k = 0; k < 4; k++) {
        int ni = c - 1 + k;
        double xi = g->x0[a] + g->h * ni, dw;
        w[k] = 0.0;
        if (ni < 0 || ni > g->nc[a]) continue;
        if (gimp_s0_1d(A, B, xi, g->h) == 0.0) continue;
        gimp_1d(A, B, xi, g->h, &w[k], &dw);
    }
    return 4;
}

/* Nodal forces of surface tractions carried by material points (the Neumann load of the strip
 * footing of Sec. 5.2, applied through the boundary points' domains): point q carries the force
 * F_q (the traction times the point's share of the loaded boundary) on the face of its domain
 * whose outward normal is the coordinate axis n_q (+-1 in one component, 0 elsewhere).  Along
 * that axis the grid's linear hat is evaluated on the face, x_a + lp_a n_a; along the other axes
 * the point's own 1D basis (hat or GIMP) distributes the force.  nrm NULL, or a zero normal: the
 * force acts through the point's own basis along every axis.  fext[nnode*dim] is accumulated. */
void or_surface_force(const or_grid* g, int shape, long np, const double* x, const double* lp,
                      const double* F, const double* nrm, double* fext) {
    int d = g->dim;
    int n1[3] = {g->nc[0] + 1, g->nc[1] + 1, d == 3 ? g->nc[2] + 1 : 1};
    for (long q = 0; q < np; q++) {
        int any = 0;
        for (int a = 0; a < d; a++) any |= F[q * d + a] != 0.0;
        if (!any) continue;
        int base[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
        double w[3][4];
        for (int a = 0; a < d; a++) {
            double xa = x[q * d + a], lpa = lp ? lp[q * d + a] : 0.0;
            double na = nrm ? nrm[q * d + a] : 0.0;
            if (fabs(na) > 0.5) {
                double e = xa + lpa * (na > 0 ? 1.0 : -1.0);
                cnt[a] = axis_weights(g, 0, a, e, 0.0, &base[a], w[a]);   /* hat on the face */
            } else {
                cnt[a] = axis_weights(g, shape, a, xa, lpa, &base[a], w[a]);
            }
        }
        for (int k2 = 0; k2 < cnt[2]; k2++)
            for (int k1 = 0; k1 < cnt[1]; k1++)
                for (int k0 = 0; k0 < cnt[0]; k0++) {
                    int kk[3] = {k0, k1, k2}, idx[3] = {0, 0, 0}, skip = 0;
                    double s = 1.0;
                    for (int a = 0; a < d; a++) {
                        idx[a] = base[a] + kk[a];
                        if (idx[a] < 0 || idx[a] >= n1[a]) skip = 1;
                        else s *= w[a][kk[a]];
                    }
                    if (skip || s == 0.0) continue;
                    long node = idx[0] + (long)n1[0] * (idx[1] + (long)n1[1] * idx[2]);
                    for (int b = 0; b < d; b++) fext[node * d + b] += s * F[q * d + b];
                }
    }
}

/* Cell sums of the projection operator for original MPM (eq. projection-operator, integrated at
 * the material points of each cell with their t_n volumes): Ve[c] = sum V, qe[c*2^d + k] =
 * sum V N_k over the points of cell c; Pi N_k = qe/Ve. */
void or_cell_proj(const or_grid* g, long np, const double* x, const double* V, double* Ve,
                  double* qe) {
    int d = g->dim, nv = 1 << d;
    int nodes[OR_MAXN];
    double S[OR_MAXN], G[OR_MAXN * 3];
    for (long q = 0; q < np; q++) {
        int c = 0, mul = 1;
        for (int a = 0; a < d; a++) {
            c += cell_of(g, a, x[q * d + a]) * mul;
            mul *= g->nc[a];
        }
        int n = or_basis(g, 0, x + q * d, NULL, nodes, S, G, NULL);
        Ve[c] += V[q];
        for (int k = 0; k < n; k++) qe[c * nv + k] += V[q] * S[k];
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Stage 2: residual and exact Jacobian at the material points                                 */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    /* nodal fields, natural node order */
    const double* U;    /* [nnode*dim] incremental displacement */
    const double* P;    /* [nnode] */
    const double* Pn;   /* [nnode] pressure at t_n (P2G) */
    const double* pdn;  /* [nnode] pdot at t_n (dynamic) */
    const double* pddn; /* [nnode] pddot at t_n (dynamic) */
    const double* vn;   /* [nnode*dim] velocity at t_n (dynamic) */
    const double* an;   /* [nnode*dim] acceleration at t_n (dynamic) */
    const double* Ve;   /* [ncell] original-MPM projection: cell volume */
    const double* qe;   /* [ncell*2^dim] original-MPM projection: cell moments */
} or_nodal;

/* Mobility kappa(J) = kappa0 k(phi)/k0 of the Kozeny-Carman law (Sec. 2.2, eq. kozeny-carman),
 * with the porosity of a skeleton of incompressible grains, phi = 1 - (1 - phi0)/J, J the volume
 * ratio to the initial configuration.  *dk = d kappa / d J by the chain rule through phi (zero
 * where phi is held at OR_PHI_MIN).  phi0 <= 0 gives the constant mobility kappa0. */
void or_mobility(double kappa0, double phi0, double J, double* k, double* dk) {
    if (!(phi0 > 0.0)) {
        *k = kappa0;
        *dk = 0.0;
        return;
    }
    double phi = 1.0 - (1.0 - phi0) / J;
    int held = phi < OR_PHI_MIN;
    if (held) phi = OR_PHI_MIN;
    double c0 = (1.0 - phi0) * (1.0 - phi0) / (phi0 * phi0 * phi0);
    double q = 1.0 - phi;
    *k = kappa0 * c0 * phi * phi * phi / (q * q);
    /* dk/dphi = kappa0 c0 [3 phi^2 / q^2 + 2 phi^3 / q^3],  dphi/dJ = (1 - phi0) / J^2 */
    double dk_dphi = kappa0 * c0 * (3.0 * phi * phi / (q * q) + 2.0 * phi * phi * phi / (q * q * q));
    *dk = held ? 0.0 : dk_dphi * (1.0 - phi0) / (J * J);
}

/* Kelvin-type viscous effective stress (Sec. 2.2): sigma'_vis = alpha_vis c : sym(l) with l the
 * velocity gradient in the current configuration (d x d, row-major).  Reading: c is the isotropic
 * elasticity tensor of the skeleton, lambda 1 (x) 1 + 2 G I, i.e. the spatial tangent of the
 * inviscid law at the undeformed state (so that the damping term can be linearized exactly).
 * Only the in-plane block is formed in plane strain. */
void or_viscous_stress(const or_mat* mt, int d, const double* l, double* s) {
    double tr = 0.0;
    for (int a = 0; a < d; a++) tr += l[a * d + a];
    for (int a = 0; a < d; a++)
        for (int b = 0; b < d; b++)
            s[a * d + b] = mt->alpha_vis * (mt->G * (l[a * d + b] + l[b * d + a]) + (a == b ? mt->lam * tr : 0.0));
}

/* Local residual r[nn*(d+1)] and local Jacobian Jl[(nn*(d+1))^2] (row-major, may be NULL) of
 * one material point.  Terms (Sec. 3.1-3.4, 4.2):
 *   R_mom_i  = -(V_n/J_n) tau' gradS_i + dv p^h gradS_i + m S_i (g - a^h)          (eq. residual-momentum)
 *   R_mass_i = dv S_i theta + dv kappa gradS_i . (grad p^h - rho_f (g - a^h))      (eq. residual-mass, darcy-law)
 *              with kappa = kappa(J), J = det(dF) det(F_n), when phi0 > 0 (eq. kozeny-carman)
 *              + tau V_n (S_i - Pi_i) sum_j (S_j - Pi_j) pdot_j                    (eq. stab-term-ppp)
 * with dF = 1 + sum U (x) grad_n S, dv = det(dF) V_n, gradS = dF^{-T} grad_n S (Sec. 3.3),
 * theta = ln(dJ)/dt (eq. implicit-euler) or div v^h with Newmark v (eq. newmark),
 * pdot from eq. p-dot-implicit-euler / p-dot-newmark.  Jacobian = exact directional
 * derivatives of the above with respect to every local U and P.
 * Returns nn (>0) or -1 if det(dF) <= 0. */
int or_particle(const or_grid* g, const or_mat* mt, const or_opt* op, const double* xp,
                const double* lpp, const double* Fn, double Vn, double mp, int cellid,
                const or_nodal* nd, int* nodes, double* r, double* Jl) {
    int d = g->dim, nv = 1 << d, nd1 = d + 1;
    double S[OR_MAXN], Gr[OR_MAXN * 3], S0[OR_MAXN], Pi[OR_MAXN];
    int nn = or_basis(g, op->shape, xp, lpp, nodes, S, Gr, S0);
    for (int k = 0; k < nn; k++) {
        if (op->shape == 1)
            Pi[k] = S0[k];
        else
            Pi[k] = (nd->Ve && nd->Ve[cellid] > 0) ? nd->qe[cellid * nv + k] / nd->Ve[cellid] : 0.0;
    }
    /* kinematics */
    double dF[9], f[9], F[9], tau[9];
    for (int i = 0; i < d; i++)
        for (int j = 0; j < d; j++) {
            double s = (i == j) ? 1.0 : 0.0;
            for (int k = 0; k < nn; k++) s += nd->U[nodes[k] * d + i] * Gr[k * d + j];
            dF[i * d + j] = s;
        }
    double dJ = det_n(d, dF);
    if (!(dJ > 0.0)) return -1;
    inv_n(d, dF, f);
    matmul_n(d, dF, Fn, F);
    or_kirchhoff(mt->model, mt->lam, mt->G, d, F, tau);
    double Jn = det_n(d, Fn);
    double V0 = Vn / Jn, dv = dJ * Vn;
    double Jt = dJ * Jn, kap, dkap;
    or_mobility(mt->kappa, mt->phi0, Jt, &kap, &dkap);
    double gS[OR_MAXN * 3];
    for (int k = 0; k < nn; k++)
        for (int a = 0; a < d; a++) {
            double s = 0;
            for (int b = 0; b < d; b++) s += f[b * d + a] * Gr[k * d + b];
            gS[k * d + a] = s;
        }
    double ph = 0, gp[3] = {0, 0, 0};
    for (int k = 0; k < nn; k++) {
        double Pk = nd->P[nodes[k]];
        ph += S[k] * Pk;
        for (int a = 0; a < d; a++) gp[a] += Pk * gS[k * d + a];
    }
    double dt = op->dt, be = op->beta, ga = op->gamma;
    double ah[3] = {0, 0, 0}, l[9] = {0}, theta;
    double vel[OR_MAXN * 3];
    if (op->dynamic) {
        for (int k = 0; k < nn; k++) {
            int i = nodes[k];
            for (int c = 0; c < d; c++) {
                double Uc = nd->U[i * d + c], v0 = nd->vn[i * d + c], a0 = nd->an[i * d + c];
                double acc = Uc / (be * dt * dt) - v0 / (be * dt) + (1.0 - 1.0 / (2.0 * be)) * a0;
                vel[k * d + c] = ga / (be * dt) * Uc + (1.0 - ga / be) * v0 + (1.0 - ga / (2.0 * be)) * dt * a0;
                ah[c] += S[k] * acc;
            }
        }
        for (int k = 0; k < nn; k++)
            for (int a = 0; a < d; a++)
                for (int b = 0; b < d; b++) l[a * d + b] += vel[k * d + a] * gS[k * d + b];
        theta = 0;
        for (int a = 0; a < d; a++) theta += l[a * d + a];
    } else {
        theta = log(dJ) / dt;
    }
    double w[3];
    for (int a = 0; a < d; a++) w[a] = gp[a] - mt->rho_f * (mt->g[a] - ah[a]);
    /* viscous stress of the Newmark velocity field (dynamic problems only, eq. quasi-static-condition) */
    int vis = op->dynamic && mt->alpha_vis != 0.0;
    double svis[9] = {0};
    if (vis) or_viscous_stress(mt, d, l, svis);
    double ct = op->dynamic ? ga / (be * dt) : 1.0 / dt;
    double pstab = 0;
    if (op->tau != 0.0) {
        for (int k = 0; k < nn; k++) {
            int i = nodes[k];
            double hk = 0;
            if (op->dynamic) hk = (1.0 - ga / be) * nd->pdn[i] + (1.0 - ga / (2.0 * be)) * dt * nd->pddn[i];
            double pdot = ct * (nd->P[i] - nd->Pn[i]) + hk;
            pstab += (S[k] - Pi[k]) * pdot;
        }
    }
    /* residual */
    for (int k = 0; k < nn; k++) {
        for (int a = 0; a < d; a++) {
            double s = 0;
            for (int b = 0; b < d; b++) s += tau[a * 3 + b] * gS[k * d + b];
            double sv = 0;
            for (int b = 0; b < d; b++) sv += svis[a * d + b] * gS[k * d + b];
            r[k * nd1 + a] = -V0 * s + dv * ph * gS[k * d + a] + mp * S[k] * (mt->g[a] - ah[a]) - dv * sv;
        }
        double dw = 0;
        for (int a = 0; a < d; a++) dw += gS[k * d + a] * w[a];
        r[k * nd1 + d] = dv * S[k] * theta + dv * kap * dw + op->tau * Vn * (S[k] - Pi[k]) * pstab;
    }
    if (!Jl) return nn;
    /* Jacobian: one column at a time */
    int nl = nn * nd1;
    for (int kb = 0; kb < nn; kb++) {
        for (int c = 0; c < d; c++) {
            int col = kb * nd1 + c;
            double L[9] = {0};
            for (int y = 0; y < d; y++) L[c * d + y] = gS[kb * d + y];
            double trL = gS[kb * d + c];
            double dtau[9];
            or_dkirchhoff(mt->model, mt->lam, mt->G, d, F, L, dtau);
            double ddv = dv * trL;
            double dah[3] = {0, 0, 0};
            if (op->dynamic) dah[c] = S[kb] / (be * dt * dt);
            double dgp[3];
            for (int y = 0; y < d; y++) dgp[y] = -gS[kb * d + y] * gp[c];
            double dth;
            if (op->dynamic) {
                dth = ga / (be * dt) * gS[kb * d + c];
                for (int x = 0; x < d; x++) dth -= l[x * d + c] * gS[kb * d + x];
            } else {
                dth = trL / dt;
            }
            double dw[3];
            for (int a = 0; a < d; a++) dw[a] = dgp[a] + mt->rho_f * dah[a];
            /* derivative of the viscous stress: dl = (gamma/(beta dt) e_c - l e_c) (x) gradS_kb */
            double dsvis[9] = {0};
            if (vis) {
                double dl[9];
                for (int x = 0; x < d; x++)
                    for (int y = 0; y < d; y++)
                        dl[x * d + y] = ((x == c ? ga / (be * dt) : 0.0) - l[x * d + c]) * gS[kb * d + y];
                or_viscous_stress(mt, d, dl, dsvis);
            }
            for (int k = 0; k < nn; k++) {
                double dgS[3];
                for (int y = 0; y < d; y++) dgS[y] = -gS[kb * d + y] * gS[k * d + c];
                for (int a = 0; a < d; a++) {
                    double s1 = 0, s2 = 0;
                    for (int b = 0; b < d; b++) {
                        s1 += dtau[a * 3 + b] * gS[k * d + b];
                        s2 += tau[a * 3 + b] * dgS[b];
                    }
                    double v = -V0 * (s1 + s2) + ddv * ph * gS[k * d + a] + dv * ph * dgS[a] - mp * S[k] * dah[a];
                    if (vis) {
                        double t1 = 0, t2 = 0, t3 = 0;
                        for (int b = 0; b < d; b++) {
                            t1 += svis[a * d + b] * gS[k * d + b];
                            t2 += dsvis[a * d + b] * gS[k * d + b];
                            t3 += svis[a * d + b] * dgS[b];
                        }
                        v -= ddv * t1 + dv * t2 + dv * t3;
                    }
                    Jl[(k * nd1 + a) * nl + col] = v;
                }
                double gw = 0, dgw = 0, gdw = 0;
                for (int a = 0; a < d; a++) {
                    gw += gS[k * d + a] * w[a];
                    dgw += dgS[a] * w[a];
                    gdw += gS[k * d + a] * dw[a];
                }
                /* d(J)/dU = J trL, so d(kappa)/dU = dkap J trL */
                double v = ddv * S[k] * theta + dv * S[k] * dth + kap * (ddv * gw + dv * dgw + dv * gdw) +
                           dkap * Jt * trL * dv * gw;
                Jl[(k * nd1 + d) * nl + col] = v;
            }
        }
        /* pressure column */
        int col = kb * nd1 + d;
        for (int k = 0; k < nn; k++) {
            for (int a = 0; a < d; a++) Jl[(k * nd1 + a) * nl + col] = dv * S[kb] * gS[k * d + a];
            double gg = 0;
            for (int a = 0; a < d; a++) gg += gS[k * d + a] * gS[kb * d + a];
            Jl[(k * nd1 + d) * nl + col] =
                dv * kap * gg + op->tau * ct * Vn * (S[k] - Pi[k]) * (S[kb] - Pi[kb]);
        }
    }
    return nn;
}

static int particle_cell(const or_grid* g, const double* xp) {
    int c = 0, mul = 1;
    for (int a = 0; a < g->dim; a++) {
        c += cell_of(g, a, xp[a]) * mul;
        mul *= g->nc[a];
    }
    return c;
}

/* Global assembly: R[nnode*(d+1)] += sum of local residuals; the Jacobian is returned as COO
 * triplets (duplicates allowed) when coo_v != NULL, and/or as the product Jv = J vin when
 * Jv != NULL.  Returns the number of COO entries, or -1 - q if particle q is inverted. */
long or_assemble(const or_grid* g, const or_mat* mt, const or_opt* op, long np, const double* x,
                 const double* lp, const double* F, const double* V, const double* m,
                 const or_nodal* nd, double* R, long* coo_i, long* coo_j, double* coo_v,
                 long coo_cap, const double* vin, double* Jv) {
    int d = g->dim, nd1 = d + 1;
    int nodes[OR_MAXN];
    double r[OR_MAXN * 4];
    int need_J = (coo_v != NULL) || (Jv != NULL);
    double* Jl = need_J ? (double*)malloc(sizeof(double) * (OR_MAXN * 4) * (OR_MAXN * 4)) : NULL;
    long cnt = 0;
    for (long q = 0; q < np; q++) {
        int nn = or_particle(g, mt, op, x + q * d, lp ? lp + q * d : NULL, F + q * d * d, V[q], m[q],
                             particle_cell(g, x + q * d), nd, nodes, r, Jl);
        if (nn < 0) {
            free(Jl);
            return -1 - q;
        }
        int nl = nn * nd1;
        for (int k = 0; k < nn; k++)
            for (int c = 0; c < nd1; c++) R[(long)nodes[k] * nd1 + c] += r[k * nd1 + c];
        if (!need_J) continue;
        for (int i = 0; i < nl; i++) {
            long gi = (long)nodes[i / nd1] * nd1 + i % nd1;
            for (int j = 0; j < nl; j++) {
                long gj = (long)nodes[j / nd1] * nd1 + j % nd1;
                double v = Jl[i * nl + j];
                if (Jv) Jv[gi] += v * vin[gj];
                if (coo_v) {
                    if (cnt < coo_cap) {
                        coo_i[cnt] = gi;
                        coo_j[cnt] = gj;
                        coo_v[cnt] = v;
                    }
                    cnt++;
                }
            }
        }
    }
    free(Jl);
    return cnt;
}

/* ------------------------------------------------------------------------------------------ */
/* Stages 3-4: nodes -> particles, convection, domain update (Sec. 3.5)                        */
/* ------------------------------------------------------------------------------------------ */

/* Right stretch tensor U = sqrt(F^T F) of a 2x2 F by the eigen-decomposition of C. */
static void right_stretch2(const double* F, double* Us) {
    double C[4] = {F[0] * F[0] + F[2] * F[2], F[0] * F[1] + F[2] * F[3], 0, F[1] * F[1] + F[3] * F[3]};
    C[2] = C[1];
    double ev[2], Q[4];
    eig_sym2(C, ev, Q);
    double s0 = sqrt(ev[0]), s1 = sqrt(ev[1]);
    for (int i = 0; i < 2; i++)
        for (int j = 0; j < 2; j++) Us[i * 2 + j] = Q[i * 2 + 0] * s0 * Q[j * 2 + 0] + Q[i * 2 + 1] * s1 * Q[j * 2 + 1];
}

/* Updates every particle from the converged nodal solution:
 *   u, x += sum S U;  F = dF F_n;  V = det(dF) V_n;  p = sum S P;  sigma' = tau'(F)/J;
 *   dynamic: v += dt sum S [(1-gamma) a_n + gamma a] (FLIP), a = sum S a, pdot/pddot = sum S of the
 *   nodal Newmark values (eq. p-dot-newmark);
 *   GIMP: lp_d = min(lp0_d U_dd, h/2) with U the right stretch of F (reading of the symmetric
 *   material stretch rule).  sig is [np*9]. Returns 0 or -1 - q on an inverted particle. */
long or_g2p(const or_grid* g, const or_mat* mt, const or_opt* op, long np, double* x, double* lp,
            const double* lp0, double* F, double* V, double* p, double* u, double* v, double* a,
            double* pd, double* pdd, double* sig, const or_nodal* nd) {
    int d = g->dim;
    int nodes[OR_MAXN];
    double S[OR_MAXN], Gr[OR_MAXN * 3];
    double dt = op->dt, be = op->beta, ga = op->gamma;
    double ct = op->dynamic ? ga / (be * dt) : 1.0 / dt;
    for (long q = 0; q < np; q++) {
        int nn = or_basis(g, op->shape, x + q * d, lp ? lp + q * d : NULL, nodes, S, Gr, NULL);
        double dF[9];
        for (int i = 0; i < d; i++)
            for (int j = 0; j < d; j++) {
                double s = (i == j) ? 1.0 : 0.0;
                for (int k = 0; k < nn; k++) s += nd->U[nodes[k] * d + i] * Gr[k * d + j];
                dF[i * d + j] = s;
            }
        double dJ = det_n(d, dF);
        if (!(dJ > 0)) return -1 - q;
        double Fnew[9];
        matmul_n(d, dF, F + q * d * d, Fnew);
        memcpy(F + q * d * d, Fnew, sizeof(double) * d * d);
        V[q] *= dJ;
        double du[3] = {0, 0, 0}, pp = 0, an[3] = {0, 0, 0}, acc[3] = {0, 0, 0}, pdq = 0, pddq = 0;
        for (int k = 0; k < nn; k++) {
            int i = nodes[k];
            pp += S[k] * nd->P[i];
            for (int c = 0; c < d; c++) du[c] += S[k] * nd->U[i * d + c];
            if (op->dynamic) {
                for (int c = 0; c < d; c++) {
                    double Uc = nd->U[i * d + c], v0 = nd->vn[i * d + c], a0 = nd->an[i * d + c];
                    double ai = Uc / (be * dt * dt) - v0 / (be * dt) + (1.0 - 1.0 / (2.0 * be)) * a0;
                    an[c] += S[k] * a0;
                    acc[c] += S[k] * ai;
                }
                double dP = nd->P[i] - nd->Pn[i];
                double pdi = ct * dP + (1.0 - ga / be) * nd->pdn[i] + (1.0 - ga / (2.0 * be)) * dt * nd->pddn[i];
                double pddi = dP / (be * dt * dt) - nd->pdn[i] / (be * dt) + (1.0 - 1.0 / (2.0 * be)) * nd->pddn[i];
                pdq += S[k] * pdi;
                pddq += S[k] * pddi;
            }
        }
        for (int c = 0; c < d; c++) {
            u[q * d + c] += du[c];
            x[q * d + c] += du[c];
        }
        p[q] = pp;
        if (op->dynamic) {
            for (int c = 0; c < d; c++) {
                v[q * d + c] += dt * ((1.0 - ga) * an[c] + ga * acc[c]);
                a[q * d + c] = acc[c];
            }
            pd[q] = pdq;
            pdd[q] = pddq;
        }
        double tau[9], J = det_n(d, Fnew);
        or_kirchhoff(mt->model, mt->lam, mt->G, d, Fnew, tau);
        for (int i = 0; i < 9; i++) sig[q * 9 + i] = tau[i] / J;
        if (op->shape == 1 && d == 2) {
            double Us[4];
            right_stretch2(Fnew, Us);
            for (int c = 0; c < 2; c++) {
                double l = lp0[q * 2 + c] * Us[c * 2 + c];
                lp[q * 2 + c] = l < 0.5 * g->h ? l : 0.5 * g->h;
            }
        }
    }
    return 0;
}
