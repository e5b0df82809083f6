// Geometric multigrid for the two sub-blocks of the block upper-triangular preconditioner of
// the Newton-Krylov solver (Sec. 3.4): family A (displacement block, dim x dim node blocks) and
// family S (scalar Schur approximation: the fixed-stress form C + C_stab + (c_t/K) M_p, whose
// level 0 is J's pressure block plus a diagonal, or the diagonal-inverse form C - B2 diag(A)^-1 B1,
// whose level 0 is stored whole).
//
// Hierarchy: the structured background grid, coarsened by two along every axis that still has
// more than three nodes (semi-coarsening keeps elongated grids solvable); bilinear/trilinear
// transfer; Galerkin coarse operators P^T A P built on the device; level-0 operators are views
// into the stored Jacobian blocks (no copy; the diagonal-inverse Schur form excepted).  Smoother: damped block Jacobi, V(nsm, nsm).
// Coarsest level: dense inverse (Gauss-Jordan in LDS, at most CMAX unknowns).
//
// Launch structure: levels with more than TAILMAX nodes use one kernel per operation (pre-smooth
// fused with the residual, restriction, prolongation, post-smooth); all smaller levels of a
// problem run inside one block of a single "tail" kernel, which removes most of the launches of
// a V-cycle.  Every kernel serves a whole batch of problems.
#include "solver_common.hpp"
#include "launch.hpp"

namespace ppm {

// 1D weight of fine node i from coarse node I: linear interpolation between the coarse
// positions min(2I, nf - 1) (the last coarse node sits on the last fine node)
__device__ __forceinline__ double pw1(int i, int I, int nf) {
    if ((i & 1) == 0) return I == (i >> 1) ? 1.0 : 0.0;
    int lo = (i - 1) >> 1, hi = lo + 1;
    int phi = min(2 * hi, nf - 1);
    if (phi == i) return I == hi ? 1.0 : 0.0;
    return (I == lo || I == hi) ? 0.5 : 0.0;
}
// same, with the identity on axes that are not coarsened
__device__ __forceinline__ double pwa(int i, int I, int nf, int cz) {
    return cz ? pw1(i, I, nf) : (i == I ? 1.0 : 0.0);
}
// k-th fine candidate (k = 0, 1, 2) of coarse index I along one axis; -1 if none
__device__ __forceinline__ int cand(int I, int k, int cz) { return cz ? 2 * I - 1 + k : (k == 1 ? I : -1); }

template <int BB>
__device__ __forceinline__ void invert_small(const double* A, double* Ai) {
    if (BB == 1) {
        Ai[0] = (A[0] == 0.0 || !isfinite(A[0])) ? 1.0 : 1.0 / A[0];
        return;
    }
    double dt = BB == 2 ? det<2>(A) : det<3>(A);
    if (dt == 0.0 || !isfinite(dt)) {
        for (int i = 0; i < BB * BB; ++i) Ai[i] = (i % (BB + 1) == 0) ? 1.0 : 0.0;
        return;
    }
    if (BB == 2) inverse<2>(A, Ai);
    else inverse<3>(A, Ai);
}

// ---------------------------------------------------------------------------------------------
// row operations (one grid node of one level).  The stencil shape (DIM, R) is a compile-time
// constant so that the stencil loops unroll and every load of a row is issued at once; the
// level's sizes and operator pointers are read once per thread into an Lv.
// ---------------------------------------------------------------------------------------------
template <typename T>
struct Lv {
    int n0, n1, n2, np0, np1;
    int64_t nrow;
    const T* op;   // operator storage (level 0: the Jacobian, row-blocked)
    int BJ, a0;    // block size of the storage, first row/column of the family inside it
    int sh;        // index = (row >> sh) * bstride + e * estride + (row & mask)
    int64_t mask, estride, bstride;
    const T* Di;   // inverse diagonal blocks
    __device__ __forceinline__ double opv(int s, int a, int c, int64_t row) const {
        const int64_t e = (int64_t)(s * BJ + a + a0) * BJ + c + a0;
        return (double)op[(row >> sh) * bstride + e * estride + (row & mask)];
    }
};

template <int BB, typename T>
__device__ __forceinline__ Lv<T> lv_of(const Dev* d, int fam, int l) {
    const MgLevel& L = d->lev[l];
    Lv<T> v;
    v.n0 = L.n[0];
    v.n1 = L.n[1];
    v.n2 = L.n[2];
    v.np0 = L.np[0];
    v.np1 = L.np[1];
    v.nrow = L.nrow;
    if (l == 0 && !(fam == 1 && d->schur)) {
        v.op = (const T*)d->J;
        v.BJ = d->b;
        v.a0 = fam == 0 ? 0 : d->dim;
        const bool blk = d->dim == 3;   // layout of jidx
        v.sh = blk ? 6 : 62;
        v.mask = blk ? (int64_t)(JB - 1) : ~(int64_t)0;
        v.estride = blk ? (int64_t)JB : d->Nnode;
        v.bstride = blk ? (int64_t)d->S * d->b * d->b * JB : 0;
    } else {
        v.op = (const T*)(fam == 0 ? L.A : L.Sm);
        v.BJ = BB;
        v.a0 = 0;
        v.sh = 62;
        v.mask = ~(int64_t)0;
        v.estride = L.nrow;
        v.bstride = 0;
    }
    v.Di = (const T*)(fam == 0 ? L.Ad : L.Sd);
    return v;
}

// real coordinates of row and its padded index
template <int DIM, int R, typename T>
__device__ __forceinline__ int64_t lv_pad(const Lv<T>& v, int64_t row, int* c) {
    c[0] = (int)(row % v.n0);
    c[1] = (int)((row / v.n0) % v.n1);
    c[2] = DIM == 3 ? (int)(row / ((int64_t)v.n0 * v.n1)) : 0;
    int64_t p = (int64_t)(c[1] + R);
    if (DIM == 3) p += (int64_t)v.np1 * (c[2] + R);
    return (int64_t)(c[0] + R) + (int64_t)v.np0 * p;
}

template <int DIM, int R>
struct Sten {
    static constexpr int SW = 2 * R + 1;
    static constexpr int S = DIM == 2 ? SW * SW : SW * SW * SW;
    static constexpr int C = (S - 1) / 2;
    static constexpr int ox(int s) { return s % SW - R; }
    static constexpr int oy(int s) { return (s / SW) % SW - R; }
    static constexpr int oz(int s) { return DIM == 3 ? s / (SW * SW) - R : 0; }
};

template <int BB, typename T>
__device__ __forceinline__ void dinv_apply(const Lv<T>& v, int64_t row, const double* x, double* out) {
#pragma unroll
    for (int a = 0; a < BB; ++a) {
        double t = 0.0;
#pragma unroll
        for (int c = 0; c < BB; ++c) t += (double)v.Di[(int64_t)(a * BB + c) * v.nrow + row] * x[c];
        out[a] = t;
    }
}

// x = omega Dinv rhs
template <int DIM, int R, int BB, typename T>
__device__ __forceinline__ void row_smooth0(const Dev* d, const Lv<T>& v, int64_t row, View<T> rhs, View<T> x) {
    int c[3];
    const int64_t pn = lv_pad<DIM, R>(v, row, c);
    double r[BB], y[BB];
#pragma unroll
    for (int a = 0; a < BB; ++a) r[a] = (double)rhs.at(pn, a);
    dinv_apply<BB>(v, row, r, y);
#pragma unroll
    for (int a = 0; a < BB; ++a) x.at(pn, a) = (T)(d->omega * y[a]);
}

// r = rhs - A x (ghost entries of x are zero, as are the operator entries that leave the grid);
// POST: the last post-smoothing sweep instead, r <- x + omega Dinv (rhs - A x) (r must not alias x)
template <int DIM, int R, int BB, typename T, bool FULL, bool POST = false>
__device__ __forceinline__ void row_resid(const Dev* d, const Lv<T>& v, bool fs0, int64_t row, View<T> rhs,
                                          View<T> x, View<T> r) {
    using St = Sten<DIM, R>;
    constexpr int SW = St::SW, NROW = St::S / SW;
    int c[3];
    const int64_t pn = lv_pad<DIM, R>(v, row, c);
    double acc[BB];
#pragma unroll
    for (int a = 0; a < BB; ++a) acc[a] = (double)rhs.at(pn, a);
#pragma unroll(FULL ? (DIM == 3 ? 3 : NROW) : 1)
    for (int t = 0; t < NROW; ++t) {
        const int oy = t % SW - R, oz = DIM == 3 ? t / SW - R : 0;
        const int64_t poff = (int64_t)v.np0 * (oy + (int64_t)v.np1 * oz);
#pragma unroll
        for (int i = 0; i < SW; ++i) {
            const int64_t pk = pn + (i - R) + poff;
            const int s = t * SW + i;
#pragma unroll
            for (int cc = 0; cc < BB; ++cc) {
                const double xv = (double)x.at(pk, cc);
#pragma unroll
                for (int a = 0; a < BB; ++a) acc[a] -= v.opv(s, a, cc, row) * xv;
            }
        }
    }
    if (fs0) acc[0] -= fs_term(d, pn) * (double)x.at(pn, 0);
    if (POST) {
        double y[BB];
        dinv_apply<BB>(v, row, acc, y);
#pragma unroll
        for (int a = 0; a < BB; ++a) r.at(pn, a) = (T)((double)x.at(pn, a) + d->omega * y[a]);
    } else {
#pragma unroll
        for (int a = 0; a < BB; ++a) r.at(pn, a) = (T)acc[a];
    }
}

// x += omega Dinv r
template <int DIM, int R, int BB, typename T>
__device__ __forceinline__ void row_update(const Dev* d, const Lv<T>& v, int64_t row, View<T> x, View<T> r) {
    int c[3];
    const int64_t pn = lv_pad<DIM, R>(v, row, c);
    double rr[BB], y[BB];
#pragma unroll
    for (int a = 0; a < BB; ++a) rr[a] = (double)r.at(pn, a);
    dinv_apply<BB>(v, row, rr, y);
#pragma unroll
    for (int a = 0; a < BB; ++a) x.at(pn, a) = (T)((double)x.at(pn, a) + d->omega * y[a]);
}

// (P^T r)_I for coarse node I[] of level l+1 (MASK: level-0 fine dofs masked by the free mask)
template <int DIM, int R, int BB, typename T, bool MASK>
__device__ __forceinline__ void restrict_gather(const Dev* d, int fam, int l, const int* I, View<T> r, double* acc) {
    const MgLevel& F = d->lev[l];
    const int fn[3] = {F.n[0], F.n[1], F.n[2]}, fz[3] = {F.cz[0], F.cz[1], F.cz[2]};
    const int fp0 = F.np[0], fp1 = F.np[1];
#pragma unroll
    for (int a = 0; a < BB; ++a) acc[a] = 0.0;
    constexpr int nI = DIM == 3 ? 27 : 9;
#pragma unroll
    for (int ii = 0; ii < nI; ++ii) {
        const int kk[3] = {ii % 3, (ii / 3) % 3, ii / 9};
        int fi[3] = {0, 0, 0};
        double w = 1.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            fi[a] = cand(I[a], kk[a], fz[a]);
            const bool ok = fi[a] >= 0 && fi[a] < fn[a];
            w = ok ? w * pwa(fi[a], I[a], fn[a], fz[a]) : 0.0;
            fi[a] = ok ? fi[a] : 0;
        }
        // no branch around the loads: a candidate off the grid was moved onto node 0 with a zero
        // weight, so all loads of the node are issued together instead of one round trip each
        int64_t fpn = (int64_t)(fi[1] + R);
        if (DIM == 3) fpn += (int64_t)fp1 * (fi[2] + R);
        fpn = (fi[0] + R) + (int64_t)fp0 * fpn;
#pragma unroll
        for (int a = 0; a < BB; ++a) {
            const double m = MASK ? mask0(d, fam, fpn, a) : 1.0;
            acc[a] += w * m * (double)r.at(fpn, a);
        }
    }
}

// the level test taken once, outside the unrolled gather (a conditional load per candidate
// would put a branch between the loads)
template <int DIM, int R, int BB, typename T>
__device__ __forceinline__ void restrict_node(const Dev* d, int fam, int l, const int* I, View<T> r, double* acc) {
    if (l == 0) restrict_gather<DIM, R, BB, T, true>(d, fam, l, I, r, acc);
    else restrict_gather<DIM, R, BB, T, false>(d, fam, l, I, r, acc);
}

// coarse rhs of node Irow on level l+1 = (P^T r)_I
template <int DIM, int R, int BB, typename T>
__device__ __forceinline__ void row_restrict(const Dev* d, int fam, int l, int64_t Irow, View<T> r, View<T> bc) {
    const MgLevel& C = d->lev[l + 1];
    int I[3];
    real_coords(Irow, C.n, DIM, I);
    double acc[BB];
    restrict_node<DIM, R, BB, T>(d, fam, l, I, r, acc);
    const int64_t cpn = padded(I, C.np, R, DIM);
#pragma unroll
    for (int a = 0; a < BB; ++a) bc.at(cpn, a) = (T)acc[a];
}

// (P xc) at fine node fi[] of level l, masked on level 0 (free dofs only)
template <int DIM, int R, int BB, typename T>
__device__ __forceinline__ void prolong_node(const Dev* d, int fam, int l, const int* fi, int64_t fpn, View<T> xc,
                                             double* acc) {
    const MgLevel& F = d->lev[l];
    const MgLevel& C = d->lev[l + 1];
    const int fn[3] = {F.n[0], F.n[1], F.n[2]}, fz[3] = {F.cz[0], F.cz[1], F.cz[2]};
    const int cn[3] = {C.n[0], C.n[1], C.n[2]};
    const int cp0 = C.np[0], cp1 = C.np[1];
#pragma unroll
    for (int a = 0; a < BB; ++a) acc[a] = 0.0;
    constexpr int nI = DIM == 3 ? 8 : 4;
#pragma unroll
    for (int jj = 0; jj < nI; ++jj) {
        int I[3] = {0, 0, 0};
        double w = 1.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int bit = (jj >> a) & 1;
            if (fz[a]) {
                I[a] = (fi[a] >> 1) + bit;
                const bool ok = I[a] < cn[a];
                w = ok ? w * pw1(fi[a], I[a], fn[a]) : 0.0;
                I[a] = ok ? I[a] : 0;
            } else {
                w = bit ? 0.0 : w;
                I[a] = fi[a];
            }
        }
        // unconditional loads (see restrict_node); I[] is a valid coarse node when w is zero
        int64_t cpn = (int64_t)(I[1] + R);
        if (DIM == 3) cpn += (int64_t)cp1 * (I[2] + R);
        cpn = (I[0] + R) + (int64_t)cp0 * cpn;
#pragma unroll
        for (int a = 0; a < BB; ++a) acc[a] += w * (double)xc.at(cpn, a);
    }
    if (l == 0) {
#pragma unroll
        for (int a = 0; a < BB; ++a) acc[a] *= mask0(d, fam, fpn, a);
    }
}

// x(fine node) += (P xc)
template <int DIM, int R, int BB, typename T>
__device__ __forceinline__ void row_prolong(const Dev* d, int fam, int l, int64_t frow, View<T> xc, View<T> x) {
    const MgLevel& F = d->lev[l];
    int fi[3];
    real_coords(frow, F.n, DIM, fi);
    const int64_t fpn = padded(fi, F.np, R, DIM);
    double acc[BB];
    prolong_node<DIM, R, BB, T>(d, fam, l, fi, fpn, xc, acc);
#pragma unroll
    for (int a = 0; a < BB; ++a) x.at(fpn, a) = (T)((double)x.at(fpn, a) + acc[a]);
}

// ---------------------------------------------------------------------------------------------
// setup kernels
// ---------------------------------------------------------------------------------------------
template <int BB, typename T>
__global__ void __launch_bounds__(TPB) k_mg_dinv(Batch B, int fam, int l) {
    PROB_PROLOGUE
    if (l >= d->nlev || (fam == 1 && l > d->ls_stop)) return;
    const MgLevel& L = d->lev[l];
    if (tid >= L.nrow) return;
    Op<T> o = op_of<T>(d, fam, l);
    const int sc = (d->S - 1) / 2;
    double A[BB * BB], Ai[BB * BB];
    for (int a = 0; a < BB; ++a)
        for (int c = 0; c < BB; ++c) A[a * BB + c] = o.at(sc, a, c, tid);
    if (fam == 1 && l == 0) {
        int cc[3];
        real_coords(tid, L.n, d->dim, cc);
        A[0] += fs_term(d, padded(cc, L.np, d->R, d->dim));
    }
    invert_small<BB>(A, Ai);
    T* out = (T*)(fam == 0 ? L.Ad : L.Sd);
    for (int k = 0; k < BB * BB; ++k) out[(int64_t)k * L.nrow + tid] = (T)Ai[k];
}

// Level-0 operator of the Schur block in the diagonal-inverse form (option schur = 1):
//   S_ij = C_ij - sum_k sum_ab B2_ik,a Dinv_k,ab B1_kj,b
// with C the pressure block of J (storage, Darcy and PPP terms), B2 its pressure-displacement and
// B1 its displacement-pressure coupling, and Dinv_k the inverse dim x dim node block of the
// displacement block (the A family's level-0 inverse diagonal, formed before this kernel).  Entry
// j of row i is taken on the Jacobian's stencil; the intermediate nodes k are those of i's stencil
// whose own stencil holds j.  Non-free displacement components drop out (their B1 rows and B2
// columns are masked); a row of a non-free pressure dof keeps J's row; columns of non-free
// pressure dofs are zero.  One thread per (row, stencil slot blockIdx.y), stored in the coarse
// levels' layout [S][nrow] in precision T.
template <int DIM, int R, typename T>
__global__ void __launch_bounds__(TPB) k_schur_diag(Batch B) {
    PROB_PROLOGUE
    if (!d->schur) return;
    const MgLevel& L = d->lev[0];
    if (tid >= L.nrow) return;
    using St = Sten<DIM, R>;
    constexpr int BS = DIM + 1, S = St::S, SW = St::SW;
    const int s = blockIdx.y;
    const T* __restrict__ J = (const T*)d->J;
    const T* __restrict__ Ad = (const T*)L.Ad;
    const int NE = S * BS * BS;
    int ci[3];
    real_coords(tid, L.n, DIM, ci);
    const int64_t pi = padded(ci, L.np, R, DIM);
    const int so[3] = {St::ox(s), St::oy(s), St::oz(s)};
    bool inj = true;
    int cj[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        cj[a] = ci[a] + so[a];
        inj = inj && cj[a] >= 0 && cj[a] < L.n[a];
    }
    double v = (double)J[jidx<DIM>((s * BS + DIM) * BS + DIM, tid, NE, d->Nnode)];
    if (mask0(d, 1, pi, 0) != 0.0) {
        if (!inj || mask0(d, 1, padded(cj, L.np, R, DIM), 0) == 0.0) {
            v = 0.0;
        } else {
            for (int t = 0; t < S; ++t) {
                const int to[3] = {St::ox(t), St::oy(t), St::oz(t)};
                int ck[3] = {0, 0, 0}, u = 0, mul = 1;
                bool ok = true;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    ck[a] = ci[a] + to[a];
                    const int du = so[a] - to[a];
                    ok = ok && ck[a] >= 0 && ck[a] < L.n[a] && du >= -R && du <= R;
                    u += (du + R) * mul;
                    mul *= SW;
                }
                if (!ok) continue;
                const int64_t k = ck[0] + (int64_t)L.n[0] * (ck[1] + (int64_t)L.n[1] * ck[2]);
                const int64_t pk = padded(ck, L.np, R, DIM);
                double c2[DIM], b1[DIM];
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    const double m = mask0(d, 0, pk, a);
                    c2[a] = m * (double)J[jidx<DIM>((t * BS + DIM) * BS + a, tid, NE, d->Nnode)];
                    b1[a] = m * (double)J[jidx<DIM>((u * BS + a) * BS + DIM, k, NE, d->Nnode)];
                }
#pragma unroll
                for (int a = 0; a < DIM; ++a)
#pragma unroll
                    for (int b = 0; b < DIM; ++b) v -= c2[a] * (double)Ad[(int64_t)(a * DIM + b) * L.nrow + k] * b1[b];
            }
        }
    }
    T* out = (T*)L.Sm;
    out[(int64_t)s * L.nrow + tid] = (T)v;
}

// Galerkin coarse operator of level l+1 (2D): thread per (coarse row, stencil entry), looping
// over the candidate pairs of the two coarse nodes
// Galerkin operator P^T A P of level l+1, one thread per (coarse node, stencil slot blockIdx.y).
// DENSE: every (i, j) candidate pair is visited with unconditional loads (a pair that leaves the
// grid or the fine stencil gets weight zero and clamped indices), so all loads can be in flight
// together: the form for small levels, whose launch is one dependent chain (2D level of 15 nodes:
// 150 -> 33 us).  Otherwise invalid pairs are skipped: on large levels, where most of the 81 pairs
// fall outside the fine stencil and occupancy hides the latency, that reads less.
template <int DIM, int BB, typename T, bool DENSE>
__global__ void __launch_bounds__(TPB) k_mg_rap(Batch B, int fam, int l) {
    PROB_PROLOGUE
    if (l + 1 >= d->nlev || (fam == 1 && l + 1 > d->ls_stop)) return;
    const MgLevel& F = d->lev[l];
    const MgLevel& C = d->lev[l + 1];
    if (tid >= C.nrow) return;
    const int s = blockIdx.y;
    const int R = d->R, SW = 2 * R + 1;
    int I[3], Jc[3] = {0, 0, 0}, off[3] = {s % SW - R, (s / SW) % SW - R, DIM == 3 ? s / (SW * SW) - R : 0};
    real_coords(tid, C.n, DIM, I);
    bool valid = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        Jc[a] = I[a] + off[a];
        if (Jc[a] < 0 || Jc[a] >= C.n[a]) valid = false;
    }
    double blk[BB * BB];
#pragma unroll
    for (int k = 0; k < BB * BB; ++k) blk[k] = 0.0;
    if (valid) {
        const Op<T> o = op_of<T>(d, fam, l);
        constexpr int nI = DIM == 3 ? 27 : 9;
        // contributions of fine candidate ii of I paired with every candidate of J
        auto row_i = [&](int ii) {
            const int ki[3] = {ii % 3, (ii / 3) % 3, ii / 9};
            int fi[3] = {0, 0, 0};
            double wi = 1.0;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                const int f = cand(I[a], ki[a], F.cz[a]);
                const bool ok = f >= 0 && f < F.n[a];
                wi = ok ? wi * pwa(f, I[a], F.n[a], F.cz[a]) : 0.0;
                fi[a] = ok ? f : 0;
            }
            if (!DENSE && wi == 0.0) return;
            const int64_t frow = fi[0] + (int64_t)F.n[0] * (fi[1] + (int64_t)F.n[1] * fi[2]);
            const int64_t fpn = padded(fi, F.np, R, DIM);
            double mi[BB];
#pragma unroll
            for (int a = 0; a < BB; ++a) mi[a] = l == 0 ? mask0(d, fam, fpn, a) : 1.0;
            auto pair = [&](int jj) {
                const int kj[3] = {jj % 3, (jj / 3) % 3, jj / 9};
                int fj[3] = {0, 0, 0};
                double w = wi;
                int fs = 0, mul = 1;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    const int f = cand(Jc[a], kj[a], F.cz[a]);
                    const int dd = f - fi[a];
                    const bool ok = f >= 0 && f < F.n[a] && dd >= -R && dd <= R;
                    w = ok ? w * pwa(f, Jc[a], F.n[a], F.cz[a]) : 0.0;
                    fj[a] = ok ? f : fi[a];
                    fs += ((ok ? dd : 0) + R) * mul;
                    mul *= SW;
                }
                if (!DENSE && w == 0.0) return;
                const int64_t fpnj = padded(fj, F.np, R, DIM);
#pragma unroll
                for (int a = 0; a < BB; ++a)
#pragma unroll
                    for (int c = 0; c < BB; ++c) {
                        const double m = l == 0 ? mi[a] * mask0(d, fam, fpnj, c) : 1.0;
                        double v = o.at(fs, a, c, frow);
                        if (fam == 1 && l == 0 && fs == (d->S - 1) / 2) v += fs_term(d, fpn);
                        blk[a * BB + c] += w * m * v;
                    }
            };
            if constexpr (DENSE) {
#pragma unroll
                for (int jj = 0; jj < nI; ++jj) pair(jj);
            } else {
                for (int jj = 0; jj < nI; ++jj) pair(jj);
            }
        };
        // (DENSE: the pairs of one fine candidate of I are issued together, candidate by
        // candidate, which keeps a row's loads within the register budget)
        for (int ii = 0; ii < nI; ++ii) row_i(ii);
        if (s == (d->S - 1) / 2)
#pragma unroll
            for (int a = 0; a < BB; ++a)
                if (blk[a * BB + a] == 0.0) blk[a * BB + a] = 1.0;
    }
    T* out = (T*)(fam == 0 ? C.A : C.Sm);
#pragma unroll
    for (int a = 0; a < BB; ++a)
#pragma unroll
        for (int c = 0; c < BB; ++c) out[((int64_t)(s * BB + a) * BB + c) * C.nrow + tid] = (T)blk[a * BB + c];
}

// Galerkin coarse operator of level l+1 (3D), one thread per (coarse row I, component pair (a, c)):
// for every fine candidate i of I (weight P_iI) and every stencil entry delta of fine row i,
// A_f(i, i + delta) goes to the coarse parents J of j = i + delta with weight P_iI P_jJ.  On a
// coarsened axis i = 2I - 1 + k and j = 2I + m with m = k + delta - 1, so the parents of j sit
// at J - I = m/2 (m even) or (m-1)/2 + {0, 1} (m odd); on other axes J = j.  Each thread owns a
// column of stencil-slot accumulators in LDS (no sharing, fixed summation order).
__device__ __forceinline__ int rap_parents(int cz, int k, int dl, int* off) {
    if (!cz) {
        off[0] = dl;
        return k == 1 ? 1 : 0;
    }
    const int m = k + dl - 1;
    if ((m & 1) == 0) {
        off[0] = m / 2;
        return 1;
    }
    off[0] = (m - 1) / 2;
    off[1] = off[0] + 1;
    return 2;
}

template <int DIM, int R, int BB, typename T>
__global__ void __launch_bounds__(TPB) k_mg_rap2(Batch B, int fam, int l) {
    constexpr int SW = 2 * R + 1;
    constexpr int S = DIM == 2 ? SW * SW : SW * SW * SW;
    __shared__ double sacc[S * TPB];
    PROB_PROLOGUE
    if (l + 1 >= d->nlev || (fam == 1 && l + 1 > d->ls_stop)) return;
    const MgLevel& F = d->lev[l];
    const MgLevel& C = d->lev[l + 1];
    if (tid >= C.nrow) return;
    const int a = blockIdx.y / BB, c = blockIdx.y % BB;
    double* acc = sacc + threadIdx.x;   // slot s at acc[s * TPB]
    for (int s = 0; s < S; ++s) acc[s * TPB] = 0.0;
    const int fn[3] = {F.n[0], F.n[1], F.n[2]}, cn[3] = {C.n[0], C.n[1], C.n[2]};
    const int cz[3] = {F.cz[0], F.cz[1], DIM == 3 ? F.cz[2] : 0};
    Op<T> o = op_of<T>(d, fam, l);
    int I[3];
    real_coords(tid, C.n, DIM, I);
    constexpr int NK = DIM == 2 ? 9 : 27;
    for (int kk = 0; kk < NK; ++kk) {
        const int k[3] = {kk % 3, (kk / 3) % 3, kk / 9};
        int fi[3] = {0, 0, 0};
        double wi = 1.0;
        for (int ax = 0; ax < DIM; ++ax) {
            if (!cz[ax] && k[ax] != 1) wi = 0.0;
            fi[ax] = cz[ax] ? 2 * I[ax] - 1 + k[ax] : I[ax];
            if (fi[ax] < 0 || fi[ax] >= fn[ax]) wi = 0.0;
            if (wi != 0.0) wi *= pwa(fi[ax], I[ax], fn[ax], cz[ax]);
        }
        if (wi == 0.0) continue;
        const int64_t frow = fi[0] + (int64_t)fn[0] * (fi[1] + (int64_t)fn[1] * fi[2]);
        const int64_t fpn = padded(fi, F.np, d->R, DIM);
        if (l == 0 && mask0(d, fam, fpn, a) == 0.0) continue;
        // the fine row's S entries (and, on level 0, the column masks) loaded together before the
        // scatter: the stored row holds zeros in the slots that leave the grid, and a ghost
        // column's mask is read inside the padded array
        double vs[S];
#pragma unroll
        for (int s = 0; s < S; ++s) vs[s] = o.at(s, a, c, frow);
        if (l == 0) {
            if (fam == 1) vs[(S - 1) / 2] += fs_term(d, fpn);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int dl[3] = {s % SW - R, (s / SW) % SW - R, DIM == 3 ? s / (SW * SW) - R : 0};
                int fj[3] = {0, 0, 0};
#pragma unroll
                for (int ax = 0; ax < DIM; ++ax) fj[ax] = fi[ax] + dl[ax];
                vs[s] *= mask0(d, fam, padded(fj, F.np, d->R, DIM), c);
            }
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int dl[3] = {s % SW - R, (s / SW) % SW - R, DIM == 3 ? s / (SW * SW) - R : 0};
            int fj[3] = {0, 0, 0};
            bool jok = true;
            for (int ax = 0; ax < DIM; ++ax) {
                fj[ax] = fi[ax] + dl[ax];
                if (fj[ax] < 0 || fj[ax] >= fn[ax]) jok = false;
            }
            if (!jok) continue;
            double v = vs[s];
            if (v == 0.0) continue;
            v *= wi;
            int off[3][2], np[3] = {1, 1, 1};
            for (int ax = 0; ax < DIM; ++ax) np[ax] = rap_parents(cz[ax], k[ax], dl[ax], off[ax]);
            for (int bz = 0; bz < (DIM == 3 ? np[2] : 1); ++bz)
                for (int by = 0; by < np[1]; ++by)
                    for (int bx = 0; bx < np[0]; ++bx) {
                        const int o3[3] = {off[0][bx], off[1][by], DIM == 3 ? off[2][bz] : 0};
                        double wj = 1.0;
                        for (int ax = 0; ax < DIM; ++ax) {
                            const int J = I[ax] + o3[ax];
                            if (J < 0 || J >= cn[ax]) wj = 0.0;
                            else if (cz[ax]) wj *= pw1(fj[ax], J, fn[ax]);
                        }
                        if (wj == 0.0) continue;
                        const int slot = (o3[0] + R) + SW * ((o3[1] + R) + (DIM == 3 ? SW * (o3[2] + R) : 0));
                        acc[slot * TPB] += wj * v;
                    }
        }
    }
    // stencil slots that leave the coarse grid hold zero; an empty row gets a unit diagonal
    T* out = (T*)(fam == 0 ? C.A : C.Sm);
    for (int s = 0; s < S; ++s) {
        const int off3[3] = {s % SW - R, (s / SW) % SW - R, DIM == 3 ? s / (SW * SW) - R : 0};
        bool valid = true;
        for (int ax = 0; ax < DIM; ++ax) {
            const int J = I[ax] + off3[ax];
            if (J < 0 || J >= cn[ax]) valid = false;
        }
        double v = valid ? acc[s * TPB] : 0.0;
        if (s == (S - 1) / 2 && a == c && v == 0.0) v = 1.0;
        out[((int64_t)(s * BB + a) * BB + c) * C.nrow + tid] = (T)v;
    }
}

// Galerkin coarse operator of level l+1 (3D) as three one-axis products.  The prolongation is a
// tensor product of 1D interpolations, P = P_x P_y P_z (each acting on one axis), so
//   R A P = P_z^T (P_y^T (P_x^T A P_x) P_y) P_z:
// pass p coarsens axis p of the rows and of the stencil offsets, on a grid whose axes before p
// are already coarse and whose axes after p are still fine.  Every operator on the way keeps the
// 27-point stencil (a 3-point coupling under linear interpolation spans 3 coarse points).  The
// two intermediates are FP64, in the scratch of the 3D cell matrices (free between the Jacobian
// gather and the next assembly); the first pass applies the level-0 dof masks and the
// fixed-stress diagonal, the last writes the level's operator (unit diagonal in empty rows).  One
// thread per (output row, component pair): 3 fine candidates x 27 slots loaded, 27 stores, where
// the single-pass product (k_mg_rap2) loads 27 x 27 per coarse row and pair.
__device__ __forceinline__ int64_t rap_axis_rows(const MgLevel& F, const MgLevel& C, int p) {
    int64_t r = 1;
    for (int ax = 0; ax < 3; ++ax) r *= ax <= p ? C.n[ax] : F.n[ax];
    return r;
}

template <int BB, typename T, bool FIRST, bool LAST>
__global__ void __launch_bounds__(TPB) k_mg_rap_axis(Batch B, int fam, int l, int p) {
    PROB_PROLOGUE
    if (l + 1 >= d->nlev || (fam == 1 && l + 1 > d->ls_stop)) return;
    const MgLevel& F = d->lev[l];
    const MgLevel& C = d->lev[l + 1];
    int gin[3], gout[3];
    for (int ax = 0; ax < 3; ++ax) {
        gin[ax] = ax < p ? C.n[ax] : F.n[ax];
        gout[ax] = ax <= p ? C.n[ax] : F.n[ax];
    }
    const int64_t nin = (int64_t)gin[0] * gin[1] * gin[2];
    const int64_t nout = (int64_t)gout[0] * gout[1] * gout[2];
    if (tid >= nout) return;
    const int a = blockIdx.y / BB, c = blockIdx.y % BB;
    double* t1 = (double*)d->Ke;   // after pass 0: [27][BB][BB][rows of pass 0]
    double* t2 = t1 + rap_axis_rows(F, C, 0) * 27 * BB * BB;   // after pass 1
    const double* src = p == 1 ? t1 : t2;
    double* dst = p == 0 ? t1 : t2;
    int O[3];
    O[0] = (int)(tid % gout[0]);
    O[1] = (int)((tid / gout[0]) % gout[1]);
    O[2] = (int)(tid / ((int64_t)gout[0] * gout[1]));
    const int cz = F.cz[p], nf = F.n[p], nc = C.n[p];
    const int stride = p == 0 ? 1 : (p == 1 ? 3 : 9);
    double acc[27];
#pragma unroll
    for (int s = 0; s < 27; ++s) acc[s] = 0.0;
    Op<T> o;
    if (FIRST) o = op_of<T>(d, fam, l);
    for (int k = 0; k < 3; ++k) {
        const int i = cand(O[p], k, cz);
        if (i < 0 || i >= nf) continue;
        const double wi = pwa(i, O[p], nf, cz);
        if (wi == 0.0) continue;
        int I[3] = {O[0], O[1], O[2]};
        I[p] = i;
        const int64_t irow = I[0] + (int64_t)gin[0] * (I[1] + (int64_t)gin[1] * I[2]);
        double v[27];
        if (FIRST) {
#pragma unroll
            for (int s = 0; s < 27; ++s) v[s] = o.at(s, a, c, irow);
            if (l == 0) {
                const int64_t ipn = padded(I, F.np, d->R, 3);
                const double rm = mask0(d, fam, ipn, a);
                if (fam == 1) v[13] += fs_term(d, ipn);
#pragma unroll
                for (int s = 0; s < 27; ++s) {
                    const int J[3] = {I[0] + s % 3 - 1, I[1] + (s / 3) % 3 - 1, I[2] + s / 9 - 1};
                    v[s] *= rm * mask0(d, fam, padded(J, F.np, d->R, 3), c);
                }
            }
        } else {
#pragma unroll
            for (int s = 0; s < 27; ++s) v[s] = src[((int64_t)(s * BB + a) * BB + c) * nin + irow];
        }
#pragma unroll
        for (int s = 0; s < 27; ++s) {
            const int dl = (s / stride) % 3 - 1;
            const int j = i + dl;
            if (j < 0 || j >= nf || v[s] == 0.0) continue;
            const double vv = wi * v[s];
            int off[2] = {0, 0};
            const int npar = rap_parents(cz, k, dl, off);
            for (int q2 = 0; q2 < npar; ++q2) {
                const int Jp = O[p] + off[q2];
                if (Jp < 0 || Jp >= nc) continue;
                const double wj = cz ? pw1(j, Jp, nf) : 1.0;
                acc[s + (off[q2] - dl) * stride] += wj * vv;
            }
        }
    }
    if (!LAST) {
#pragma unroll
        for (int s = 0; s < 27; ++s) dst[((int64_t)(s * BB + a) * BB + c) * nout + tid] = acc[s];
        return;
    }
    T* out = (T*)(fam == 0 ? C.A : C.Sm);
#pragma unroll
    for (int s = 0; s < 27; ++s) {
        const int J[3] = {O[0] + s % 3 - 1, O[1] + (s / 3) % 3 - 1, O[2] + s / 9 - 1};
        const bool valid = J[0] >= 0 && J[1] >= 0 && J[2] >= 0 && J[0] < C.n[0] && J[1] < C.n[1] && J[2] < C.n[2];
        double w = valid ? acc[s] : 0.0;
        if (s == 13 && a == c && w == 0.0) w = 1.0;
        out[((int64_t)(s * BB + a) * BB + c) * C.nrow + tid] = (T)w;
    }
}

// Dense inverse of the coarsest operator, Gauss-Jordan with partial pivoting in FP64 in LDS,
// one block per problem (n <= CMAX).
template <int BB, typename T>
__global__ void __launch_bounds__(256) k_mg_coarse_setup(Batch B, int fam) {
    const int q = blockIdx.x;
    const Dev* d = B.d[q];
    const int l = d->nlev - 1;
    const MgLevel& L = d->lev[l];
    const int dim = d->dim, R = d->R;
    const int n = (int)(L.nrow * BB);
    if (n > CMAX || (fam == 1 && d->ls_stop < d->ltail)) return;
    __shared__ double M[CMAX][CMAX + 1];
    __shared__ int perm[CMAX];
    __shared__ int piv;
    Op<T> o = op_of<T>(d, fam, l);
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) M[e / n][e % n] = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) perm[i] = i;
    __syncthreads();
    for (int e = threadIdx.x; e < L.nrow * d->S; e += blockDim.x) {
        int64_t row = e % L.nrow;
        int s = (int)(e / L.nrow);
        int c0[3], c1[3] = {0, 0, 0};
        real_coords(row, L.n, dim, c0);
        const int SW = 2 * R + 1;
        int off[3] = {s % SW - R, (s / SW) % SW - R, dim == 3 ? s / (SW * SW) - R : 0};
        bool ok = true;
        for (int a = 0; a < dim; ++a) {
            c1[a] = c0[a] + off[a];
            if (c1[a] < 0 || c1[a] >= L.n[a]) ok = false;
        }
        if (!ok) continue;
        int64_t col = c1[0] + (int64_t)L.n[0] * (c1[1] + (int64_t)L.n[1] * c1[2]);
        for (int a = 0; a < BB; ++a)
            for (int c = 0; c < BB; ++c) {
                double v = o.at(s, a, c, row);
                if (fam == 1 && l == 0 && s == (d->S - 1) / 2) v += fs_term(d, padded(c0, L.np, R, dim));
                M[row * BB + a][col * BB + c] = v;
            }
    }
    __syncthreads();
    static_assert(CMAX <= 128, "one thread per column and half the rows below");
    const int cc = threadIdx.x & 127, rh = threadIdx.x >> 7;
    for (int k = 0; k < n; ++k) {
        if (threadIdx.x < 64) {
            // partial pivoting: largest |M[r][k]|, r >= k (the lowest row on ties), found by the
            // first wavefront with a shuffle reduction
            int best = -1;
            double bv = -1.0;
            for (int r = k + (int)threadIdx.x; r < n; r += 64) {
                const double v = fabs(M[r][k]);
                if (v > bv) { bv = v; best = r; }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const double ov = __shfl_xor(bv, o);
                const int ob = __shfl_xor(best, o);
                if (ov > bv || (ov == bv && ob >= 0 && (best < 0 || ob < best))) { bv = ov; best = ob; }
            }
            if (threadIdx.x == 0) piv = best < 0 ? k : best;
        }
        __syncthreads();
        const int pr = piv;
        if (pr != k) {
            for (int c = threadIdx.x; c < n; c += blockDim.x) {
                double t = M[k][c]; M[k][c] = M[pr][c]; M[pr][c] = t;
            }
            if (threadIdx.x == 0) { int t = perm[k]; perm[k] = perm[pr]; perm[pr] = t; }
        }
        __syncthreads();
        double pv = M[k][k];
        if (pv == 0.0 || !isfinite(pv)) pv = 1.0;
        // row k scaled by 1/pv off the diagonal; the diagonal takes 1/pv after the barrier, during
        // the elimination, which reads neither it nor column k of row k
        for (int c = threadIdx.x; c < n; c += blockDim.x)
            if (c != k) M[k][c] /= pv;
        __syncthreads();
        if (threadIdx.x == 0) M[k][k] = 1.0 / pv;
        if (cc < n && cc != k) {
            const double mkc = M[k][cc];
#pragma unroll 8
            for (int r = rh; r < n; r += 2)
                if (r != k) M[r][cc] -= M[r][k] * mkc;
        }
        __syncthreads();
        for (int r = threadIdx.x; r < n; r += blockDim.x)
            if (r != k) M[r][k] = -M[r][k] * M[k][k];
        __syncthreads();
    }
    // the row swaps of the factorization permute the columns of the inverse
    T* out = (T*)(fam == 0 ? d->cinvA : d->cinvS);
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        int r = e / n, c = e % n;
        out[(int64_t)r * n + perm[c]] = (T)M[r][c];
    }
}

// ---------------------------------------------------------------------------------------------
// cycle kernels of the large levels (one thread per row, batched)
// ---------------------------------------------------------------------------------------------
template <int DIM, int R, int BB, typename T>
__global__ void __launch_bounds__(TPB) k_mg_smooth0(Batch B, int fam, int l, VRef rv, VRef xv) {
    PROB_PROLOGUE
    if (krylov_done(d) || l >= d->ltail || tid >= d->lev[l].nrow) return;
    const Lv<T> v = lv_of<BB, T>(d, fam, l);
    row_smooth0<DIM, R, BB, T>(d, v, tid, resolve<T>(d, rv, fam, l, BB), resolve<T>(d, xv, fam, l, BB));
}

template <int DIM, int R, int BB, typename T, bool FULL>
__global__ void __launch_bounds__(TPB) k_mg_resid(Batch B, int fam, int l, VRef rv, VRef xv, VRef resv) {
    PROB_PROLOGUE
    if (krylov_done(d) || l >= d->ltail || tid >= d->lev[l].nrow) return;
    const Lv<T> v = lv_of<BB, T>(d, fam, l);
    row_resid<DIM, R, BB, T, FULL>(d, v, fam == 1 && l == 0, tid, resolve<T>(d, rv, fam, l, BB),
                             resolve<T>(d, xv, fam, l, BB), resolve<T>(d, resv, fam, l, BB));
}

template <int DIM, int R, int BB, typename T, bool FULL>
__global__ void __launch_bounds__(TPB) k_mg_post(Batch B, int fam, int l, VRef rv, VRef xv, VRef outv) {
    PROB_PROLOGUE
    if (krylov_done(d) || l >= d->ltail || tid >= d->lev[l].nrow) return;
    const Lv<T> v = lv_of<BB, T>(d, fam, l);
    row_resid<DIM, R, BB, T, FULL, true>(d, v, fam == 1 && l == 0, tid, resolve<T>(d, rv, fam, l, BB),
                                         resolve<T>(d, xv, fam, l, BB), resolve<T>(d, outv, fam, l, BB));
}

template <int DIM, int R, int BB, typename T>
__global__ void __launch_bounds__(TPB) k_mg_update(Batch B, int fam, int l, VRef xv, VRef resv) {
    PROB_PROLOGUE
    if (krylov_done(d) || l >= d->ltail || tid >= d->lev[l].nrow) return;
    const Lv<T> v = lv_of<BB, T>(d, fam, l);
    row_update<DIM, R, BB, T>(d, v, tid, resolve<T>(d, xv, fam, l, BB), resolve<T>(d, resv, fam, l, BB));
}

template <int DIM, int R, int BB, typename T>
__global__ void __launch_bounds__(TPB) k_mg_restrict(Batch B, int fam, int l, VRef rv, VRef bv) {
    PROB_PROLOGUE
    // the transfer into the first tail level is done by the tail kernel
    if (krylov_done(d) || l + 1 >= d->ltail || l + 1 >= d->nlev || (fam == 1 && l + 1 > d->ls_stop) ||
        tid >= d->lev[l + 1].nrow)
        return;
    row_restrict<DIM, R, BB, T>(d, fam, l, tid, resolve<T>(d, rv, fam, l, BB), resolve<T>(d, bv, fam, l + 1, BB));
}

template <int DIM, int R, int BB, typename T>
__global__ void __launch_bounds__(TPB) k_mg_prolong(Batch B, int fam, int l, VRef xcv, VRef xv) {
    PROB_PROLOGUE
    if (krylov_done(d) || l >= d->ltail || l + 1 >= d->nlev || tid >= d->lev[l].nrow) return;
    row_prolong<DIM, R, BB, T>(d, fam, l, tid, resolve<T>(d, xcv, fam, l + 1, BB), resolve<T>(d, xv, fam, l, BB));
}

// ---------------------------------------------------------------------------------------------
// Halo-tiled sweeps for V(1,1): one kernel per level on the way down and one on the way up.
// A block owns a tile of the level (64 x 4 or 64 x 2 x 2 nodes: a wavefront is one x-run of 64
// nodes, so it reads each operator stream in one contiguous run; 3D 32 x 4 x 2 tiles measured 8%
// slower) and first fills LDS with x0 for the tile plus a halo of R nodes (component-major,
// conflict-free; the rhs of the own node is read again from memory rather than kept in LDS, which
// halves the LDS of the down sweep), then each thread finishes its node from LDS:
//   down:  b = the level's rhs (on levels >= 1, P^T r_fine written before by k_mg_restrict, one
//          thread per coarse node), x0 = omega Dinv b in LDS, then r = b - A x0 for the tile
//          (x0 and r written);
//   up:    x' = x0 + P x_coarse in LDS, then out = x' + omega Dinv (b - A x') for the tile.
// Halo nodes are computed by both neighbouring blocks (same inputs, same values); only the
// owning block writes them.
// ---------------------------------------------------------------------------------------------
template <int DIM, int R>
struct Tile {
    static constexpr int TX = DIM == 2 ? MGT2X : MGT3X;
    static constexpr int TY = DIM == 2 ? MGT2Y : MGT3Y;
    static constexpr int TZ = DIM == 2 ? 1 : MGT3Z;
    static constexpr int HX = TX + 2 * R, HY = TY + 2 * R, HZ = DIM == 2 ? 1 : TZ + 2 * R;
    static constexpr int NS = HX * HY * HZ;
    static_assert(TX * TY * TZ == TPB, "one thread per tile node");
};

template <int DIM>
__device__ __forceinline__ void tile_origin(int64_t tile, int n0, int n1, int* o) {
    constexpr int TX = DIM == 2 ? MGT2X : MGT3X, TY = DIM == 2 ? MGT2Y : MGT3Y, TZ = DIM == 2 ? 1 : MGT3Z;
    const int ntx = (n0 + TX - 1) / TX, nty = (n1 + TY - 1) / TY;
    o[0] = (int)(tile % ntx) * TX;
    o[1] = (int)((tile / ntx) % nty) * TY;
    o[2] = DIM == 3 ? (int)(tile / ((int64_t)ntx * nty)) * TZ : 0;
}

// level node of LDS slot j (tile origin o); false when it lies off the level grid
template <int DIM, int R, typename T>
__device__ __forceinline__ bool slot_node(const Lv<T>& v, const int* o, int j, int* c) {
    using Tl = Tile<DIM, R>;
    c[0] = o[0] + j % Tl::HX - R;
    c[1] = o[1] + (j / Tl::HX) % Tl::HY - R;
    c[2] = DIM == 3 ? o[2] + j / (Tl::HX * Tl::HY) - R : 0;
    bool in = (unsigned)c[0] < (unsigned)v.n0 && (unsigned)c[1] < (unsigned)v.n1;
    if (DIM == 3) in = in && (unsigned)c[2] < (unsigned)v.n2;
    return in;
}

template <int DIM, int R, typename T>
__device__ __forceinline__ int64_t level_pad(const Lv<T>& v, const int* c) {
    int64_t p = (int64_t)(c[1] + R);
    if (DIM == 3) p += (int64_t)v.np1 * (c[2] + R);
    return (int64_t)(c[0] + R) + (int64_t)v.np0 * p;
}

// thread's own node: LDS slot, level coordinates; false when off the grid
template <int DIM, int R, typename T>
__device__ __forceinline__ bool own_node(const Lv<T>& v, const int* o, int* c, int* slot) {
    using Tl = Tile<DIM, R>;
    const int t = threadIdx.x;
    const int tx = t % Tl::TX, ty = (t / Tl::TX) % Tl::TY, tz = DIM == 3 ? t / (Tl::TX * Tl::TY) : 0;
    c[0] = o[0] + tx;
    c[1] = o[1] + ty;
    c[2] = o[2] + tz;
    *slot = (tx + R) + Tl::HX * ((ty + R) + (DIM == 3 ? Tl::HY * (tz + R) : 0));
    bool in = c[0] < v.n0 && c[1] < v.n1;
    if (DIM == 3) in = in && c[2] < v.n2;
    return in;
}

// Operator row of a thread's own node.  PRE (coarse levels, rows of at most 100 entries): loaded
// into registers at kernel start, so that its latency overlaps the halo loads instead of following
// the barrier; otherwise read from memory where it is used.
template <int DIM, int R, int BB, typename T, bool PRE>
struct OwnRow {
    static constexpr int N = PRE ? Sten<DIM, R>::S * BB * BB : 1;
    T w[N];
    __device__ __forceinline__ void load(const Lv<T>& v, int64_t row) {
        if constexpr (PRE) {
#pragma unroll
            for (int s = 0; s < Sten<DIM, R>::S; ++s)
#pragma unroll
                for (int a = 0; a < BB; ++a)
#pragma unroll
                    for (int c = 0; c < BB; ++c) w[(s * BB + a) * BB + c] = (T)v.opv(s, a, c, row);
        }
    }
    __device__ __forceinline__ double at(const Lv<T>& v, int s, int a, int c, int64_t row) const {
        if constexpr (PRE) return (double)w[(s * BB + a) * BB + c];
        else return v.opv(s, a, c, row);
    }
};
template <int DIM, int R, int BB, bool FULL>
constexpr bool own_row_pre() { return FULL && Sten<DIM, R>::S * BB * BB <= 100; }

// acc -= sum_s A(s) xs[slot + offset(s)], the stencil walked per x-row (FULL, or scalar blocks,
// whose rows hold few loads each: rows unrolled)
template <int DIM, int R, int BB, typename T, bool FULL, bool PRE>
__device__ __forceinline__ void lds_stencil(const Lv<T>& v, const OwnRow<DIM, R, BB, T, PRE>& orow, int64_t row,
                                            const double* xs, int slot, double* acc) {
    using Tl = Tile<DIM, R>;
    using St = Sten<DIM, R>;
    constexpr int SW = St::SW, NROW = St::S / SW;
    constexpr int UNR = BB == 1 ? NROW : (FULL ? (DIM == 3 ? 3 : NROW) : 1);
#pragma unroll(UNR)
    for (int t = 0; t < NROW; ++t) {
        const int oy = t % SW - R, oz = DIM == 3 ? t / SW - R : 0;
        const int srow = slot + Tl::HX * (oy + Tl::HY * oz);
#pragma unroll
        for (int i = 0; i < SW; ++i) {
            const int s = t * SW + i;
            const int sk = srow + i - R;
#pragma unroll
            for (int cc = 0; cc < BB; ++cc) {
                const double xv = xs[cc * Tl::NS + sk];
#pragma unroll
                for (int a = 0; a < BB; ++a) acc[a] -= orow.at(v, s, a, cc, row) * xv;
            }
        }
    }
}

// Coarse levels (FULL) launch a few blocks only: the occupancy hint lets the compiler keep all of
// a thread's operator loads in flight instead of trading registers for waves it never gets
// (3D coarse down-sweep 91 -> 22 us).
template <int DIM, int R, int BB, typename T, bool FULL>
__global__ void __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(1, FULL ? 2 : 8))) k_mg_down(Batch B, int fam, int l, VRef rhsv) {
    using Tl = Tile<DIM, R>;
    const int q = batch_find(B, blockIdx.x);
    const Dev* __restrict__ d = B.d[q];
    const int64_t tile = blockIdx.x - B.pfx[q];
    if (krylov_done(d) || l >= d->ltail || (fam == 1 && l > d->ls_stop)) return;
    __shared__ double sx[Tl::NS * BB];
    const Lv<T> v = lv_of<BB, T>(d, fam, l);
    View<T> rhs = resolve<T>(d, rhsv, fam, l, BB);
    View<T> x = resolve<T>(d, VRef{VK_LX, 0}, fam, l, BB);
    View<T> r = resolve<T>(d, VRef{VK_LR, 0}, fam, l, BB);
    int o[3];
    tile_origin<DIM>(tile, v.n0, v.n1, o);
    const double om = d->omega;
    constexpr bool PRE = own_row_pre<DIM, R, BB, FULL>();
    int c[3], slot;
    const bool own = own_node<DIM, R>(v, o, c, &slot);
    const int64_t row = c[0] + (int64_t)v.n0 * (c[1] + (int64_t)v.n1 * c[2]);
    const int64_t pn = own ? level_pad<DIM, R>(v, c) : 0;
    OwnRow<DIM, R, BB, T, PRE> orow;
    double acc[BB];
#pragma unroll
    for (int a = 0; a < BB; ++a) acc[a] = 0.0;
    if (own) {
        orow.load(v, row);
#pragma unroll
        for (int a = 0; a < BB; ++a) acc[a] = (double)rhs.at(pn, a);
    }
    // all slots of a thread unrolled, so that their loads are in flight together
#pragma unroll
    for (int jj = 0; jj < (Tl::NS + TPB - 1) / TPB; ++jj) {
        const int j = threadIdx.x + jj * TPB;
        if (j >= Tl::NS) break;
        int c[3];
        double bk[BB], xk[BB];
#pragma unroll
        for (int a = 0; a < BB; ++a) bk[a] = xk[a] = 0.0;
        if (slot_node<DIM, R>(v, o, j, c)) {
            const int64_t pn = level_pad<DIM, R>(v, c);
#pragma unroll
            for (int a = 0; a < BB; ++a) bk[a] = (double)rhs.at(pn, a);
            const int64_t row = c[0] + (int64_t)v.n0 * (c[1] + (int64_t)v.n1 * c[2]);
            dinv_apply<BB>(v, row, bk, xk);
#pragma unroll
            for (int a = 0; a < BB; ++a) xk[a] = (double)(T)(om * xk[a]);
        }
#pragma unroll
        for (int a = 0; a < BB; ++a) {
            sx[a * Tl::NS + j] = xk[a];
        }
    }
    __syncthreads();
    if (!own) return;
    lds_stencil<DIM, R, BB, T, FULL>(v, orow, row, sx, slot, acc);
    if (fam == 1 && l == 0) acc[0] -= fs_term(d, pn) * sx[slot];
#pragma unroll
    for (int a = 0; a < BB; ++a) {
        x.at(pn, a) = (T)sx[a * Tl::NS + slot];
        r.at(pn, a) = (T)acc[a];
    }
}

// ZERO: the iterate is omega Dinv rhs, formed here (a Schur cycle that ends on level 0 is two
// Jacobi sweeps from zero, one launch instead of the level's down and up kernels).
template <int DIM, int R, int BB, typename T, bool FULL, bool ZERO = false>
__global__ void __launch_bounds__(TPB) __attribute__((amdgpu_waves_per_eu(1, FULL ? 2 : 8))) k_mg_up(Batch B, int fam, int l, VRef rhsv, VRef outv) {
    using Tl = Tile<DIM, R>;
    const int q = batch_find(B, blockIdx.x);
    const Dev* __restrict__ d = B.d[q];
    const int64_t tile = blockIdx.x - B.pfx[q];
    if (krylov_done(d) || l >= d->ltail || (fam == 1 && l > d->ls_stop)) return;
    // last level of a truncated Schur hierarchy: no coarser correction, so that the down and up
    // kernels of this level are two damped Jacobi sweeps
    const bool coarse = !(fam == 1 && l == d->ls_stop);
    __shared__ double sx[Tl::NS * BB];
    const Lv<T> v = lv_of<BB, T>(d, fam, l);
    View<T> rhs = resolve<T>(d, rhsv, fam, l, BB);
    View<T> x = resolve<T>(d, VRef{VK_LX, 0}, fam, l, BB);
    View<T> xc = resolve<T>(d, VRef{VK_SOL, 0}, fam, l + 1, BB);
    View<T> out = resolve<T>(d, outv, fam, l, BB);
    int o[3];
    tile_origin<DIM>(tile, v.n0, v.n1, o);
    constexpr bool PRE = own_row_pre<DIM, R, BB, FULL>();
    int c[3], slot;
    const bool own = own_node<DIM, R>(v, o, c, &slot);
    const int64_t row = c[0] + (int64_t)v.n0 * (c[1] + (int64_t)v.n1 * c[2]);
    const int64_t pn = own ? level_pad<DIM, R>(v, c) : 0;
    OwnRow<DIM, R, BB, T, PRE> orow;
    double acc[BB];
#pragma unroll
    for (int a = 0; a < BB; ++a) acc[a] = 0.0;
    if (own) {
        orow.load(v, row);
#pragma unroll
        for (int a = 0; a < BB; ++a) acc[a] = (double)rhs.at(pn, a);
    }
#pragma unroll
    for (int jj = 0; jj < (Tl::NS + TPB - 1) / TPB; ++jj) {
        const int j = threadIdx.x + jj * TPB;
        if (j >= Tl::NS) break;
        int c[3];
        double xk[BB];
#pragma unroll
        for (int a = 0; a < BB; ++a) xk[a] = 0.0;
        if (slot_node<DIM, R>(v, o, j, c)) {
            const int64_t pn = level_pad<DIM, R>(v, c);
            if constexpr (ZERO) {
                // as the down sweep forms (and stores in precision T) its first iterate
                double bk[BB];
#pragma unroll
                for (int a = 0; a < BB; ++a) bk[a] = (double)rhs.at(pn, a);
                const int64_t srow = c[0] + (int64_t)v.n0 * (c[1] + (int64_t)v.n1 * c[2]);
                dinv_apply<BB>(v, srow, bk, xk);
#pragma unroll
                for (int a = 0; a < BB; ++a) xk[a] = (double)(T)(d->omega * xk[a]);
            } else {
                double pc[BB];
#pragma unroll
                for (int a = 0; a < BB; ++a) pc[a] = 0.0;
                if (coarse) prolong_node<DIM, R, BB, T>(d, fam, l, c, pn, xc, pc);
                // the iterate is stored in precision T after the prolongation
#pragma unroll
                for (int a = 0; a < BB; ++a) xk[a] = (double)(T)((double)x.at(pn, a) + pc[a]);
            }
        }
#pragma unroll
        for (int a = 0; a < BB; ++a) sx[a * Tl::NS + j] = xk[a];
    }
    __syncthreads();
    if (!own) return;
    double y[BB];
    lds_stencil<DIM, R, BB, T, FULL>(v, orow, row, sx, slot, acc);
    if (fam == 1 && l == 0) acc[0] -= fs_term(d, pn) * sx[slot];
    dinv_apply<BB>(v, row, acc, y);
#pragma unroll
    for (int a = 0; a < BB; ++a) out.at(pn, a) = (T)(sx[a * Tl::NS + slot] + d->omega * y[a]);
}

constexpr int TAIL_TPB = 256;

// Residual of the n rows of a tail level: r = rhs - A x (POST: out = x + omega Dinv (rhs - A x)),
// one thread per row.  (Splitting a row's stencil over several threads when the level has fewer
// rows than threads measured no faster.)
template <int DIM, int R, int BB, typename T, bool POST>
__device__ __forceinline__ void tail_resid(const Dev* d, const Lv<T>& v, bool fs0, View<T> rhs, View<T> x,
                                           View<T> out) {
    for (int64_t i = threadIdx.x; i < v.nrow; i += blockDim.x)
        row_resid<DIM, R, BB, T, true, POST>(d, v, fs0, i, rhs, x, out);
    __syncthreads();
}

// All levels from the problem's ltail down to the coarsest and back up, in one block, starting
// with the restriction of the residual of level ltail-1.  Same conventions as the per-level
// kernels: on the way down a level's iterate is in LX and its residual in LR; on the way up the
// prolongation adds the coarser correction (VK_SOL) into LX and the last smoothing sweep writes
// the level's correction to LR (level 0: to out0).
template <int DIM, int R, int BB, typename T>
__global__ void __launch_bounds__(TAIL_TPB) k_mg_tail(Batch B, int fam, VRef rhs0, VRef out0) {
    const int q = blockIdx.x;
    const Dev* d = B.d[q];
    if (krylov_done(d) || (fam == 1 && d->ls_stop < d->ltail)) return;
    const int L0 = d->ltail, L = d->nlev, nsm = d->mg_nsm;
    const VRef LX{VK_LX, 0}, LR{VK_LR, 0}, LB{VK_LB, 0}, SOL{VK_SOL, 0};
    const int nt = blockDim.x;
    // Warm this CU's L2 with the operators and inverse diagonals of the first two tail levels (or
    // the dense coarsest inverse, when the second is the coarsest), which the passes below would
    // otherwise fetch from HBM one dependent round trip at a time: one dword per 128-byte line,
    // all issued before the first restriction (offsets clamped into each array) and consumed
    // after it.
    constexpr int PF = 8;
    uint32_t pfv[4][PF];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int l = L0 + (m >> 1);
        const bool ok = l >= 1 && l < L - 1;   // level 0 is a view of the Jacobian
        const bool dense = m == 2 && l == L - 1;
        const MgLevel& Q = d->lev[ok ? l : L0];
        const int64_t nc = d->lev[L - 1].nrow * BB;
        const void* p = dense ? (fam == 0 ? d->cinvA : d->cinvS)
                              : (m & 1) ? (fam == 0 ? Q.Ad : Q.Sd) : (fam == 0 ? Q.A : Q.Sm);
        const int64_t words = ok ? ((m & 1) ? Q.nrow : Q.nrow * d->S) * BB * BB * (int64_t)sizeof(T) / 4
                                 : dense && nc <= CMAX ? nc * nc * (int64_t)sizeof(T) / 4 : 0;
        const uint32_t* base = words > 0 ? (const uint32_t*)p : (const uint32_t*)d->scal;
        const int64_t last = words > 0 ? words - 1 : 0;
#pragma unroll
        for (int j = 0; j < PF; ++j) {
            const int64_t w = ((int64_t)j * nt + threadIdx.x) * 32;
            pfv[m][j] = base[w < last ? w : last];
        }
    }
    if (L0 > 0) {
        // right-hand side of the first tail level from the residual of the level above it
        View<T> rf = resolve<T>(d, LR, fam, L0 - 1, BB);
        View<T> bc = resolve<T>(d, LB, fam, L0, BB);
        const int64_t nc = d->lev[L0].nrow;
        for (int64_t i = threadIdx.x; i < nc; i += nt) row_restrict<DIM, R, BB, T>(d, fam, L0 - 1, i, rf, bc);
        __syncthreads();
    }
    {
        uint32_t pf = 0;
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int j = 0; j < PF; ++j) pf ^= pfv[m][j];
        asm volatile("" ::"v"(pf));   // keeps the warming loads (no instruction)
    }
    for (int l = L0; l < L - 1; ++l) {
        const Lv<T> v = lv_of<BB, T>(d, fam, l);
        const bool fs0 = fam == 1 && l == 0;
        View<T> rhs = resolve<T>(d, l == 0 ? rhs0 : LB, fam, l, BB);
        View<T> x = resolve<T>(d, LX, fam, l, BB);
        View<T> r = resolve<T>(d, LR, fam, l, BB);
        const int64_t n = v.nrow;
        // smoothing from a zero guess, then the residual against the stored iterate (in one block
        // the iterate is L2-resident; the fused form would rebuild omega Dinv b for every
        // neighbour of a row)
        for (int64_t i = threadIdx.x; i < n; i += nt) row_smooth0<DIM, R, BB, T>(d, v, i, rhs, x);
        __syncthreads();
        for (int k = 1; k < nsm; ++k) {
            tail_resid<DIM, R, BB, T, false>(d, v, fs0, rhs, x, r);
            for (int64_t i = threadIdx.x; i < n; i += nt) row_update<DIM, R, BB, T>(d, v, i, x, r);
            __syncthreads();
        }
        tail_resid<DIM, R, BB, T, false>(d, v, fs0, rhs, x, r);
        View<T> bc = resolve<T>(d, LB, fam, l + 1, BB);
        const int64_t nc = d->lev[l + 1].nrow;
        for (int64_t i = threadIdx.x; i < nc; i += nt) row_restrict<DIM, R, BB, T>(d, fam, l, i, r, bc);
        __syncthreads();
    }
    {
        const int l = L - 1;
        const MgLevel& C = d->lev[l];
        View<T> rhs = resolve<T>(d, l == 0 ? rhs0 : LB, fam, l, BB);
        View<T> x = resolve<T>(d, l == 0 ? out0 : LX, fam, l, BB);
        const int n = (int)(C.nrow * BB);
        const T* Ci = (const T*)(fam == 0 ? d->cinvA : d->cinvS);
        // x = Ci b: NPART threads per row, each a fixed-length slice of the row with its loads
        // unconditional (index clamped, weight zero past n), partial sums added in LDS
        constexpr int NPART = TAIL_TPB / CMAX, SL = (CMAX + NPART - 1) / NPART;
        __shared__ double bv[CMAX + SL * NPART];
        __shared__ double part[NPART * CMAX];
        if (n <= CMAX) {
            for (int e = threadIdx.x; e < CMAX + SL * NPART; e += nt) {
                double b = 0.0;
                if (e < n) {
                    int c[3];
                    real_coords(e / BB, C.n, DIM, c);
                    b = (double)rhs.at(padded(c, C.np, R, DIM), e % BB);
                }
                bv[e] = b;
            }
            __syncthreads();
            const int e = threadIdx.x % CMAX, pi = threadIdx.x / CMAX;
            if (pi < NPART && e < n) {
                const T* crow = Ci + (int64_t)e * n;
                double t = 0.0;
#pragma unroll
                for (int j = 0; j < SL; ++j) {
                    const int k = pi * SL + j;
                    t += (double)crow[k < n ? k : n - 1] * bv[k];
                }
                part[pi * CMAX + e] = t;
            }
            __syncthreads();
            for (int e2 = threadIdx.x; e2 < n; e2 += nt) {
                double t = 0.0;
#pragma unroll
                for (int q2 = 0; q2 < NPART; ++q2) t += part[q2 * CMAX + e2];
                int c[3];
                real_coords(e2 / BB, C.n, DIM, c);
                x.at(padded(c, C.np, R, DIM), e2 % BB) = (T)t;
            }
        }
        __syncthreads();
    }
    for (int l = L - 2; l >= L0; --l) {
        const Lv<T> v = lv_of<BB, T>(d, fam, l);
        const bool fs0 = fam == 1 && l == 0;
        View<T> rhs = resolve<T>(d, l == 0 ? rhs0 : LB, fam, l, BB);
        View<T> x = resolve<T>(d, LX, fam, l, BB);
        View<T> r = resolve<T>(d, LR, fam, l, BB);
        View<T> out = resolve<T>(d, l == 0 ? out0 : LR, fam, l, BB);
        View<T> xc = resolve<T>(d, SOL, fam, l + 1, BB);
        const int64_t n = v.nrow;
        for (int64_t i = threadIdx.x; i < n; i += nt) row_prolong<DIM, R, BB, T>(d, fam, l, i, xc, x);
        __syncthreads();
        for (int k = 1; k < nsm; ++k) {
            tail_resid<DIM, R, BB, T, false>(d, v, fs0, rhs, x, r);
            for (int64_t i = threadIdx.x; i < n; i += nt) row_update<DIM, R, BB, T>(d, v, i, x, r);
            __syncthreads();
        }
        tail_resid<DIM, R, BB, T, true>(d, v, fs0, rhs, x, out);
    }
}

// t_u = y_u - B1 z_p on level 0 (B1 = displacement rows, pressure columns of J)
// Block count of the coupling product: 2D FP64 one wavefront per (component a, run of 64
// nodes), as the SpMV (16.2 -> 14.6 us on the 2D footing); otherwise one thread per node with all
// components (the split measured slower in 3D: 142 -> 160 us).
inline int64_t b1_blocks(int dim, int64_t nnode, bool fp64) {
    if (!fp64 || dim == 3) return (nnode + TPB - 1) / TPB;
    return ((nnode + 63) / 64 * dim + 3) / 4;
}

// t = y_u - B1 z_p (rhs of the displacement cycle)
template <int DIM, int R, typename T>
__global__ void __launch_bounds__(TPB) k_b1(Batch B, VRef yv, VRef zv) {
    PROB_PROLOGUE
    constexpr bool SPLIT = sizeof(T) == 8 && DIM == 2;
    constexpr int NA = SPLIT ? 1 : DIM;   // components per thread
    int a0 = 0;
    int64_t row = tid;
    if (SPLIT) {
        const int64_t W = lb * (TPB / 64) + threadIdx.x / 64;
        a0 = (int)(W % DIM);
        row = (W / DIM) * 64 + (threadIdx.x & 63);
    }
    if (krylov_done(d) || row >= d->Nnode) return;
    using St = Sten<DIM, R>;
    View<T> y = resolve<T>(d, yv, 0, 0, DIM), z = resolve<T>(d, zv, 0, 0, 1);
    View<T> t = resolve<T>(d, VRef{VK_BT, 0}, 0, 0, DIM);
    constexpr int bs = DIM + 1;
    int c[3];
    real_coords(row, d->nn, DIM, c);
    const int64_t pn = padded(c, d->np1, R, DIM);
    const int np0 = d->np1[0], np1 = d->np1[1];
    const T* J = (const T*)d->J;
    double acc[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) acc[i] = (double)y.at(pn, a0 + i);
#pragma unroll
    for (int s = 0; s < St::S; ++s) {
        const int64_t pk = pn + St::ox(s) + (int64_t)np0 * (St::oy(s) + (int64_t)np1 * St::oz(s));
        const double zp = (double)z.at(pk, 0);
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const T* jp = &J[jidx<DIM>((s * bs + a0 + i) * bs + DIM, row, St::S * bs * bs, d->Nnode)];
            // 3D: streamed from HBM as in the SpMV
            acc[i] -= (double)(DIM == 3 ? __builtin_nontemporal_load(jp) : *jp) * zp;
        }
    }
#pragma unroll
    for (int i = 0; i < NA; ++i) t.at(pn, a0 + i) = (T)acc[i];
}
// ---------------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------------
static std::vector<int64_t> level_rows(const std::vector<const Dev*>& hc, int l) {
    std::vector<int64_t> v;
    for (auto* h : hc) v.push_back(l < h->nlev ? h->lev[l].nrow : 1);
    return v;
}

// rows of pass p of the one-axis Galerkin products from level l (3D)
static int64_t rap_axis_rows_host(const Dev* h, int l, int p) {
    int64_t r = 1;
    for (int ax = 0; ax < 3; ++ax) r *= ax <= p ? h->lev[l + 1].n[ax] : h->lev[l].n[ax];
    return r;
}

// the two FP64 intermediates of the one-axis products from level l fit every problem's cell-matrix
// scratch
static bool rap_axis_fits(const std::vector<const Dev*>& hc, int l) {
    for (auto* h : hc) {
        if (h->dim != 3 || !h->Ke) return false;
        if (l + 1 >= h->nlev) continue;
        const size_t need = (size_t)(rap_axis_rows_host(h, l, 0) + rap_axis_rows_host(h, l, 1)) * 27 * 9 * sizeof(double);
        const size_t have = (size_t)h->Ncell * 16 * 64 * (h->mixed ? sizeof(float) : sizeof(double));
        if (need > have) return false;
    }
    return true;
}

static int max_levels(const std::vector<const Dev*>& hc) {
    int L = 0;
    for (auto* h : hc) L = std::max(L, h->nlev);
    return L;
}

static int max_ltail(const std::vector<const Dev*>& hc) {
    int L = 0;
    for (auto* h : hc) L = std::max(L, h->ltail);
    return L;
}

static bool any_schur(const std::vector<const Dev*>& hc) {
    for (auto* h : hc)
        if (h->schur) return true;
    return false;
}

template <int DIM, int R, typename T>
static void precond_setup_t(const Group& g, const std::vector<const Dev*>& hc, bool coarse, hipStream_t st) {
    if (!coarse) {
        // later Newton iterations of a step: the fine level follows the new Jacobian (its operator
        // is a view of J, its inverse diagonal is rebuilt here); the coarse levels are kept
        Batch Bl = make_batch(g.ddev, level_rows(hc, 0), TPB);
        hipLaunchKernelGGL((k_mg_dinv<DIM, T>), dim3(Bl.pfx[Bl.n]), dim3(TPB), 0, st, Bl, 0, 0);
        if (any_schur(hc))
            hipLaunchKernelGGL((k_schur_diag<DIM, R, T>), dim3(Bl.pfx[Bl.n], g.S), dim3(TPB), 0, st, Bl);
        hipLaunchKernelGGL((k_mg_dinv<1, T>), dim3(Bl.pfx[Bl.n]), dim3(TPB), 0, st, Bl, 1, 0);
        return;
    }
    const int Lmax = max_levels(hc);
    // deepest level of the Schur hierarchy over the batch (truncated hierarchies stop at ls_stop)
    int LmaxS = 0;
    bool full_s = false;
    for (auto* h : hc) {
        if (h->ls_stop < h->ltail) LmaxS = std::max(LmaxS, h->ls_stop + 1);
        else {
            LmaxS = std::max(LmaxS, h->nlev);
            full_s = true;
        }
    }
    for (int l = 0; l < Lmax; ++l) {
        // the coarse operator of level l is needed before its inverse diagonal
        if (l > 0) {
            Batch Bc = make_batch(g.ddev, level_rows(hc, l), TPB);
            if constexpr (DIM == 2) {
                const std::vector<int64_t> rows = level_rows(hc, l);
                if (*std::max_element(rows.begin(), rows.end()) > 4096)
                    PPM_TIMED(KT_RAP, st, hipLaunchKernelGGL((k_mg_rap<DIM, DIM, T, false>), dim3(Bc.pfx[Bc.n], g.S), dim3(TPB), 0, st, Bc, 0, l - 1));
                else
                    PPM_TIMED(KT_RAP, st, hipLaunchKernelGGL((k_mg_rap<DIM, DIM, T, true>), dim3(Bc.pfx[Bc.n], g.S), dim3(TPB), 0, st, Bc, 0, l - 1));
                if (l < LmaxS) {
                    if (*std::max_element(rows.begin(), rows.end()) > 4096)
                        hipLaunchKernelGGL((k_mg_rap<DIM, 1, T, false>), dim3(Bc.pfx[Bc.n], g.S), dim3(TPB), 0, st, Bc, 1, l - 1);
                    else
                        hipLaunchKernelGGL((k_mg_rap<DIM, 1, T, true>), dim3(Bc.pfx[Bc.n], g.S), dim3(TPB), 0, st, Bc, 1, l - 1);
                }
            } else {
                // 3D: three one-axis products through the cell-matrix scratch on every level
                // (level 0 -> 1 on the 96^3 footing: 11.1 -> 2.3 ms; the 2,197-row level 0.59 ms
                // -> three short launches); the single-pass forms remain for a scratch too small
                const std::vector<int64_t> rows = level_rows(hc, l);
                if (rap_axis_fits(hc, l - 1)) {
                    Batch Bp[3];
                    for (int p = 0; p < 3; ++p) {
                        std::vector<int64_t> r;
                        for (auto* h : hc) r.push_back(l < h->nlev ? rap_axis_rows_host(h, l - 1, p) : 1);
                        Bp[p] = make_batch(g.ddev, r, TPB);
                    }
                    const dim3 g0(Bp[0].pfx[Bp[0].n], DIM * DIM), g1(Bp[1].pfx[Bp[1].n], DIM * DIM),
                        g2(Bp[2].pfx[Bp[2].n], DIM * DIM), tb(TPB);
                    PPM_TIMED(KT_RAP, st, hipLaunchKernelGGL((k_mg_rap_axis<DIM, T, true, false>), g0, tb, 0, st, Bp[0], 0, l - 1, 0));
                    PPM_TIMED(KT_RAP, st, hipLaunchKernelGGL((k_mg_rap_axis<DIM, T, false, false>), g1, tb, 0, st, Bp[1], 0, l - 1, 1));
                    PPM_TIMED(KT_RAP, st, hipLaunchKernelGGL((k_mg_rap_axis<DIM, T, false, true>), g2, tb, 0, st, Bp[2], 0, l - 1, 2));
                    if (l < LmaxS) {
                        const dim3 h0(Bp[0].pfx[Bp[0].n], 1), h1(Bp[1].pfx[Bp[1].n], 1), h2(Bp[2].pfx[Bp[2].n], 1);
                        hipLaunchKernelGGL((k_mg_rap_axis<1, T, true, false>), h0, tb, 0, st, Bp[0], 1, l - 1, 0);
                        hipLaunchKernelGGL((k_mg_rap_axis<1, T, false, false>), h1, tb, 0, st, Bp[1], 1, l - 1, 1);
                        hipLaunchKernelGGL((k_mg_rap_axis<1, T, false, true>), h2, tb, 0, st, Bp[2], 1, l - 1, 2);
                    }
                } else if (*std::max_element(rows.begin(), rows.end()) > 4096) {
                    PPM_TIMED(KT_RAP, st, hipLaunchKernelGGL((k_mg_rap2<DIM, R, DIM, T>), dim3(Bc.pfx[Bc.n], DIM * DIM), dim3(TPB), 0, st, Bc, 0, l - 1));
                    if (l < LmaxS) hipLaunchKernelGGL((k_mg_rap2<DIM, R, 1, T>), dim3(Bc.pfx[Bc.n], 1), dim3(TPB), 0, st, Bc, 1, l - 1);
                } else {
                    PPM_TIMED(KT_RAP, st, hipLaunchKernelGGL((k_mg_rap<DIM, DIM, T, false>), dim3(Bc.pfx[Bc.n], g.S), dim3(TPB), 0, st, Bc, 0, l - 1));
                    if (l < LmaxS) hipLaunchKernelGGL((k_mg_rap<DIM, 1, T, true>), dim3(Bc.pfx[Bc.n], g.S), dim3(TPB), 0, st, Bc, 1, l - 1);
                }
            }
        }
        Batch Bl = make_batch(g.ddev, level_rows(hc, l), TPB);
        hipLaunchKernelGGL((k_mg_dinv<DIM, T>), dim3(Bl.pfx[Bl.n]), dim3(TPB), 0, st, Bl, 0, l);
        // the diagonal-inverse Schur operator needs the A family's level-0 inverse blocks
        if (l == 0 && any_schur(hc))
            hipLaunchKernelGGL((k_schur_diag<DIM, R, T>), dim3(Bl.pfx[Bl.n], g.S), dim3(TPB), 0, st, Bl);
        if (l < LmaxS) hipLaunchKernelGGL((k_mg_dinv<1, T>), dim3(Bl.pfx[Bl.n]), dim3(TPB), 0, st, Bl, 1, l);
    }
    Batch B1 = make_batch_one_block(g.ddev);
    hipLaunchKernelGGL((k_mg_coarse_setup<DIM, T>), dim3(B1.n), dim3(256), 0, st, B1, 0);
    if (full_s) hipLaunchKernelGGL((k_mg_coarse_setup<1, T>), dim3(B1.n), dim3(256), 0, st, B1, 1);
}

void launch_precond_setup(const Group& g, const std::vector<const Dev*>& hc, bool coarse, hipStream_t st) {
    if (g.dim == 2 && g.shape == 0) {
        if (g.mixed) precond_setup_t<2, 1, float>(g, hc, coarse, st);
        else precond_setup_t<2, 1, double>(g, hc, coarse, st);
    } else if (g.dim == 2) {
        if (g.mixed) precond_setup_t<2, 2, float>(g, hc, coarse, st);
        else precond_setup_t<2, 2, double>(g, hc, coarse, st);
    } else {
        if (g.mixed) precond_setup_t<3, 1, float>(g, hc, coarse, st);
        else precond_setup_t<3, 1, double>(g, hc, coarse, st);
    }
}

// Down-sweep of one level with nsm >= 2 sweeps (per-operation kernels): pre-smoothing from a
// zero guess (iterate -> LX, residual -> LR) and restriction of the residual to the next level's
// right-hand side.
template <int DIM, int R, int BB, typename T, bool FULL>
static void vcycle_down(const Group& g, const std::vector<const Dev*>& hc, int fam, int l, VRef rhs, int nsm,
                        hipStream_t st) {
    const VRef LX{VK_LX, 0}, LR{VK_LR, 0}, LB{VK_LB, 0};
    Batch Bl = make_batch(g.ddev, level_rows(hc, l), TPB);
    const dim3 gl(Bl.pfx[Bl.n]), tb(TPB);
    hipLaunchKernelGGL((k_mg_smooth0<DIM, R, BB, T>), gl, tb, 0, st, Bl, fam, l, rhs, LX);
    for (int k = 1; k < nsm; ++k) {
        hipLaunchKernelGGL((k_mg_resid<DIM, R, BB, T, FULL>), gl, tb, 0, st, Bl, fam, l, rhs, LX, LR);
        hipLaunchKernelGGL((k_mg_update<DIM, R, BB, T>), gl, tb, 0, st, Bl, fam, l, LX, LR);
    }
    PPM_TIMED((l == 0 ? (fam == 0 ? KT_MG0_RESID : KT_MG0_S) : -1), st,
              hipLaunchKernelGGL((k_mg_resid<DIM, R, BB, T, FULL>), gl, tb, 0, st, Bl, fam, l, rhs, LX, LR));
    Batch Bc = make_batch(g.ddev, level_rows(hc, l + 1), TPB);
    hipLaunchKernelGGL((k_mg_restrict<DIM, R, BB, T>), dim3(Bc.pfx[Bc.n]), tb, 0, st, Bc, fam, l, LR, LB);
}

// Up-sweep of one level: LX += P (coarser correction), post-smoothing, the last sweep fused with
// the residual and written to `out` (LR, or the Krylov output on level 0).
template <int DIM, int R, int BB, typename T, bool FULL>
static void vcycle_up(const Group& g, const std::vector<const Dev*>& hc, int fam, int l, VRef rhs, VRef out, int nsm,
                      hipStream_t st) {
    const VRef LX{VK_LX, 0}, LR{VK_LR, 0}, SOL{VK_SOL, 0};
    Batch Bl = make_batch(g.ddev, level_rows(hc, l), TPB);
    const dim3 gl(Bl.pfx[Bl.n]), tb(TPB);
    hipLaunchKernelGGL((k_mg_prolong<DIM, R, BB, T>), gl, tb, 0, st, Bl, fam, l, SOL, LX);
    for (int k = 1; k < nsm; ++k) {
        hipLaunchKernelGGL((k_mg_resid<DIM, R, BB, T, FULL>), gl, tb, 0, st, Bl, fam, l, rhs, LX, LR);
        hipLaunchKernelGGL((k_mg_update<DIM, R, BB, T>), gl, tb, 0, st, Bl, fam, l, LX, LR);
    }
    PPM_TIMED((l == 0 ? (fam == 0 ? KT_MG0_RESID : KT_MG0_S) : -1), st,
              hipLaunchKernelGGL((k_mg_post<DIM, R, BB, T, FULL>), gl, tb, 0, st, Bl, fam, l, rhs, LX, out));
}


// 3D displacement block: levels 0 .. ROW_LEVELS_3D - 1 are swept row by row, the others by halo
// tiles (see vcycle)
constexpr int ROW_LEVELS_3D = 2;

static std::vector<int64_t> level_tiles(const std::vector<const Dev*>& hc, int l) {
    std::vector<int64_t> v;
    for (auto* h : hc) v.push_back(l < h->nlev ? mg_tiles(h->dim, h->lev[l].n) : 1);
    return v;
}

// One batched V-cycle of family fam (block BB): rhs0 / out0 are the level-0 Krylov references.
// V(1,1): one halo-tiled kernel per level and direction; the fine level walks its stencil row by
// row (occupancy hides latency there), the coarser levels unroll it (their grids cover a few CUs
// only).  More smoothing sweeps use the per-operation kernels.
template <int DIM, int R, int BB, typename T>
static void vcycle(const Group& g, const std::vector<const Dev*>& hc, int fam, VRef rhs0, VRef out0, int nsm,
                   hipStream_t st) {
    int Lstd = max_ltail(hc);
    bool need_tail = true;
    if (fam == 1) {
        // truncated Schur hierarchies end at ls_stop (down and up there, no tail)
        int L = 0;
        need_tail = false;
        for (auto* h : hc) {
            if (h->ls_stop < h->ltail) L = std::max(L, h->ls_stop + 1);
            else {
                L = std::max(L, h->ltail);
                need_tail = true;
            }
        }
        Lstd = L;
    }
    const VRef LR{VK_LR, 0}, LB{VK_LB, 0}, LX{VK_LX, 0};
    const dim3 tb(TPB);
    if (fam == 1 && nsm == 1) {
        bool level0 = true;
        for (auto* h : hc) level0 = level0 && h->ls_stop == 0;
        if (level0) {
            Batch Bt = make_batch_blocks(g.ddev, level_tiles(hc, 0));
            PPM_TIMED(KT_MG0_S, st,
                      hipLaunchKernelGGL((k_mg_up<DIM, R, BB, T, false, true>), dim3(Bt.pfx[Bt.n]), tb, 0, st, Bt, fam, 0,
                                         rhs0, out0));
            return;
        }
    }
    // 3D displacement block, finest level: row sweeps instead of the halo tile (a 64 x 2 x 2 tile
    // forms omega Dinv b for 66 x 4 x 4 slots, 4.1 per node, and its operator streams start off
    // the 64-row blocks of the Jacobian; the row kernels read the operator in whole blocks and the
    // neighbours' iterates through L2: HBM bytes 1.35x -> 1.05x the algorithmic ones, FP64 step
    // 330 -> 320 ms, FP32 176 -> 166 ms on the 96^3 footing).  In 2D the tile halo is 1.5 nodes
    // per node and the two extra launches of the row form cost more than they save (512 x 256
    // footing: 31.6 -> 32.3 ms per FP64 step).  The first coarse level (120k rows on the 96^3
    // footing) gains from the row form too (FP64 step 293 -> 288 ms, mixed 130 -> 128); the
    // second no longer does.
    const int nrows = DIM == 3 && fam == 0 ? ROW_LEVELS_3D : 0;   // levels swept row by row
    if (nsm == 1) {
        for (int l = 0; l < Lstd; ++l) {
            Batch Bt = make_batch_blocks(g.ddev, level_tiles(hc, l));
            const dim3 gt(Bt.pfx[Bt.n]);
            if (l < nrows) {
                // also restricts to level l + 1
                if (l == 0) vcycle_down<DIM, R, BB, T, false>(g, hc, fam, 0, rhs0, 1, st);
                else vcycle_down<DIM, R, BB, T, true>(g, hc, fam, l, LB, 1, st);
            } else if (l == 0) {
                PPM_TIMED(fam == 0 ? KT_MG0_RESID : KT_MG0_S, st,
                          hipLaunchKernelGGL((k_mg_down<DIM, R, BB, T, false>), gt, tb, 0, st, Bt, fam, 0, rhs0));
            } else {
                // restriction of the finer residual once per coarse node, then the sweep reads it
                Batch Bc = make_batch(g.ddev, level_rows(hc, l), TPB);
                if (l != nrows)
                    hipLaunchKernelGGL((k_mg_restrict<DIM, R, BB, T>), dim3(Bc.pfx[Bc.n]), tb, 0, st, Bc, fam, l - 1, LR,
                                       LB);
                hipLaunchKernelGGL((k_mg_down<DIM, R, BB, T, true>), gt, tb, 0, st, Bt, fam, l, LB);
            }
        }
    } else {
        for (int l = 0; l < Lstd; ++l) {
            if (l == 0) vcycle_down<DIM, R, BB, T, false>(g, hc, fam, l, rhs0, nsm, st);
            else vcycle_down<DIM, R, BB, T, true>(g, hc, fam, l, LB, nsm, st);
        }
    }
    Batch B1 = make_batch_one_block(g.ddev);
    if (need_tail)
        hipLaunchKernelGGL((k_mg_tail<DIM, R, BB, T>), dim3(B1.n), dim3(TAIL_TPB), 0, st, B1, fam, rhs0, out0);
    if (nsm == 1) {
        for (int l = Lstd - 1; l >= 0; --l) {
            Batch Bt = make_batch_blocks(g.ddev, level_tiles(hc, l));
            const dim3 gt(Bt.pfx[Bt.n]);
            if (l < nrows) {
                if (l == 0) vcycle_up<DIM, R, BB, T, false>(g, hc, fam, 0, rhs0, out0, 1, st);
                else vcycle_up<DIM, R, BB, T, true>(g, hc, fam, l, LB, LR, 1, st);
            } else if (l == 0)
                PPM_TIMED(fam == 0 ? KT_MG0_RESID : KT_MG0_S, st,
                          hipLaunchKernelGGL((k_mg_up<DIM, R, BB, T, false>), gt, tb, 0, st, Bt, fam, 0, rhs0, out0));
            else
                hipLaunchKernelGGL((k_mg_up<DIM, R, BB, T, true>), gt, tb, 0, st, Bt, fam, l, LB, LR);
        }
    } else {
        for (int l = Lstd - 1; l >= 0; --l) {
            if (l == 0) vcycle_up<DIM, R, BB, T, false>(g, hc, fam, l, rhs0, out0, nsm, st);
            else vcycle_up<DIM, R, BB, T, true>(g, hc, fam, l, LB, LR, nsm, st);
        }
    }
    (void)LX;
}

// z = P^-1 y on Krylov vectors iy -> iz: Schur block first, then A
template <int DIM, int R, typename T>
static void precond_apply_t(const Group& g, const std::vector<const Dev*>& hc, int iy, int iz, hipStream_t st) {
    const int nsm = hc[0]->mg_nsm;
    vcycle<DIM, R, 1, T>(g, hc, 1, VRef{iy, DIM}, VRef{iz, DIM}, nsm, st);
    std::vector<int64_t> nb;
    for (size_t q = 0; q < g.nnode.size(); ++q) nb.push_back(b1_blocks(DIM, g.nnode[q], sizeof(T) == 8));
    Batch Bn = make_batch_blocks(g.ddev, nb);
    hipLaunchKernelGGL((k_b1<DIM, R, T>), dim3(Bn.pfx[Bn.n]), dim3(TPB), 0, st, Bn, VRef{iy, 0}, VRef{iz, DIM});
    vcycle<DIM, R, DIM, T>(g, hc, 0, VRef{VK_BT, 0}, VRef{iz, 0}, nsm, st);
}

void launch_precond_apply(const Group& g, const std::vector<const Dev*>& hc, int iy, int iz, hipStream_t st) {
    if (g.dim == 2 && g.shape == 0) {
        if (g.mixed) precond_apply_t<2, 1, float>(g, hc, iy, iz, st);
        else precond_apply_t<2, 1, double>(g, hc, iy, iz, st);
    } else if (g.dim == 2) {
        if (g.mixed) precond_apply_t<2, 2, float>(g, hc, iy, iz, st);
        else precond_apply_t<2, 2, double>(g, hc, iy, iz, st);
    } else {
        if (g.mixed) precond_apply_t<3, 1, float>(g, hc, iy, iz, st);
        else precond_apply_t<3, 1, double>(g, hc, iy, iz, st);
    }
}

}  // namespace ppm
