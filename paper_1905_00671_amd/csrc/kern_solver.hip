// Linear solver of each Newton iteration (Sec. 3.4): BiCGStab on the fixed-stencil block rows
// of the Jacobian, right-preconditioned by the block upper-triangular operator
//       P = [ A  B1 ]      applied as   z_p = S^-1 r_p,   z_u = A^-1 (r_u - B1 z_p)
//           [ 0  S  ]
// (the Schur complement first, then A, as in the paper's solver).  The inverses are one
// geometric-multigrid V-cycle each on the structured background grid: damped block-Jacobi
// smoothing, bilinear transfer, Galerkin coarse operators R A P built on the device, a dense
// inverse on the coarsest level.  S is approximated by the fixed-stress form
// C + C_stab + (c_t / K) M_p (M_p lumped, K = lam + 2G/dim).
//
// Precision T is double (FP64 path) or float (mixed path: Jacobian, SpMV, preconditioner and
// Krylov vectors in FP32; dot products accumulate in FP64; the Newton update is FP64).
// Every BiCGStab scalar stays on the device; a per-problem flag stops finished problems.
#include "ppmpm_internal.hpp"
#include "launch.hpp"

namespace ppm {

#define PROB_PROLOGUE                                   \
    const int q = batch_find(B, blockIdx.x);            \
    const Dev* __restrict__ d = B.d[q];                 \
    const int64_t lb = blockIdx.x - B.pfx[q];           \
    const int64_t tid = lb * blockDim.x + threadIdx.x;

template <typename T> __device__ __forceinline__ T* vp(void* p) { return (T*)p; }

__device__ __forceinline__ void real_coords(int64_t row, const int* n, int dim, int* c) {
    c[0] = (int)(row % n[0]);
    c[1] = (int)((row / n[0]) % n[1]);
    c[2] = dim == 3 ? (int)(row / ((int64_t)n[0] * n[1])) : 0;
}
__device__ __forceinline__ int64_t padded(const int* c, const int* np, int R, int dim) {
    if (dim == 2) return (int64_t)(c[0] + R) + (int64_t)np[0] * (c[1] + R);
    return (int64_t)(c[0] + R) + (int64_t)np[0] * ((c[1] + R) + (int64_t)np[1] * (c[2] + R));
}
__device__ __forceinline__ int64_t stencil_offset(int s, int R, int dim, const int* np) {
    int SW = 2 * R + 1;
    int dx = s % SW - R, dy = (s / SW) % SW - R, dz = dim == 3 ? s / (SW * SW) - R : 0;
    return (int64_t)dx + (int64_t)np[0] * (dy + (int64_t)np[1] * dz);
}

// block reduction of up to 3 values into partial[lb*4 + k]
template <int NV>
__device__ __forceinline__ void block_partials(const Dev* d, int64_t lb, const double* v) {
    __shared__ double sh[NV][TPB];
    for (int k = 0; k < NV; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int off = TPB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int k = 0; k < NV; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < NV; ++k) d->partial[lb * 4 + k] = sh[k][0];
}

__device__ __forceinline__ bool krylov_done(const Dev* d) { return d->scal[SC_DONE] != 0.0; }

// ---------------------------------------------------------------------------------------------
// SpMV on the fixed-stencil block rows: y = J x, optional dot products
//   mode 1: partial (a, y)        mode 2: partials (y, a), (y, y)
// ---------------------------------------------------------------------------------------------
template <int DIM, int R, typename T>
__global__ void __launch_bounds__(TPB) k_spmv(Batch B, int ix, int iy, int ia, int mode, int check_done) {
    PROB_PROLOGUE
    constexpr int BS = DIM + 1;
    constexpr int SW = 2 * R + 1;
    constexpr int S = DIM == 2 ? SW * SW : SW * SW * SW;
    double dots[2] = {0.0, 0.0};
    bool skip = check_done && krylov_done(d);
    if (!skip && tid < d->Nnode) {
        void* const vecs[10] = {d->kx, d->kr, d->kh, d->kp, d->kv, d->ks, d->kt, d->kph, d->ksh, d->kbt};
        const T* __restrict__ x = vp<T>(vecs[ix]);
        T* __restrict__ y = vp<T>(vecs[iy]);
        const T* __restrict__ J = vp<T>(d->J);
        const int64_t Nn = d->Nnode;
        int c[3];
        real_coords(tid, d->nn, DIM, c);
        const int64_t pn = padded(c, d->np1, R, DIM);
        double acc[BS];
        for (int a = 0; a < BS; ++a) acc[a] = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int64_t pk = pn + stencil_offset(s, R, DIM, d->np1);
            T xv[BS];
#pragma unroll
            for (int cc = 0; cc < BS; ++cc) xv[cc] = x[pk * BS + cc];
#pragma unroll
            for (int a = 0; a < BS; ++a) {
                T t = 0;
#pragma unroll
                for (int cc = 0; cc < BS; ++cc) t += J[((int64_t)(s * BS + a) * BS + cc) * Nn + tid] * xv[cc];
                acc[a] += (double)t;
            }
        }
        for (int a = 0; a < BS; ++a) y[pn * BS + a] = (T)acc[a];
        if (mode) {
            const T* __restrict__ av = vp<T>(vecs[ia]);
            for (int a = 0; a < BS; ++a) {
                double yv = (double)(T)acc[a];
                dots[0] += (double)av[pn * BS + a] * yv;
                dots[1] += yv * yv;
            }
        }
    }
    if (mode) block_partials<2>(d, lb, dots);
}

// ---------------------------------------------------------------------------------------------
// BiCGStab vector kernels (thread per real node, b dofs each)
// ---------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ int64_t node_pad(const Dev* d, int64_t tid) {
    int c[3];
    real_coords(tid, d->nn, d->dim, c);
    return padded(c, d->np1, d->R, d->dim);
}

// x = 0, r = rhat = -R, p = v = 0; partial (r, r)
template <typename T>
__global__ void __launch_bounds__(TPB) k_bicg_init(Batch B) {
    PROB_PROLOGUE
    double v[1] = {0.0};
    if (tid < d->Nnode) {
        const int64_t pn = node_pad<T>(d, tid);
        const int bs = d->b;
        for (int a = 0; a < bs; ++a) {
            int64_t k = pn * bs + a;
            T r = (T)(-d->Rv[k]);
            vp<T>(d->kx)[k] = 0;
            vp<T>(d->kr)[k] = r;
            vp<T>(d->kh)[k] = r;
            vp<T>(d->kp)[k] = 0;
            vp<T>(d->kv)[k] = 0;
            v[0] += (double)r * (double)r;
        }
    }
    block_partials<1>(d, lb, v);
}

// p = r + beta (p - omega v)
template <typename T>
__global__ void __launch_bounds__(TPB) k_bicg_p(Batch B) {
    PROB_PROLOGUE
    if (krylov_done(d) || tid >= d->Nnode) return;
    const int64_t pn = node_pad<T>(d, tid);
    const int bs = d->b;
    const T beta = (T)d->scal[SC_BETA], om = (T)d->scal[SC_OMEGA];
    for (int a = 0; a < bs; ++a) {
        int64_t k = pn * bs + a;
        T* p = vp<T>(d->kp);
        p[k] = vp<T>(d->kr)[k] + beta * (p[k] - om * vp<T>(d->kv)[k]);
    }
}

// s = r - alpha v; partial (s, s)
template <typename T>
__global__ void __launch_bounds__(TPB) k_bicg_s(Batch B) {
    PROB_PROLOGUE
    double v[1] = {0.0};
    if (!krylov_done(d) && tid < d->Nnode) {
        const int64_t pn = node_pad<T>(d, tid);
        const int bs = d->b;
        const T al = (T)d->scal[SC_ALPHA];
        for (int a = 0; a < bs; ++a) {
            int64_t k = pn * bs + a;
            T sv = vp<T>(d->kr)[k] - al * vp<T>(d->kv)[k];
            vp<T>(d->ks)[k] = sv;
            v[0] += (double)sv * (double)sv;
        }
    }
    block_partials<1>(d, lb, v);
}

// x += alpha ph + omega sh; r = s - omega t; partials (rhat, r), (r, r)
template <typename T>
__global__ void __launch_bounds__(TPB) k_bicg_xr(Batch B) {
    PROB_PROLOGUE
    double v[2] = {0.0, 0.0};
    if (!krylov_done(d) && tid < d->Nnode) {
        const int64_t pn = node_pad<T>(d, tid);
        const int bs = d->b;
        const T al = (T)d->scal[SC_ALPHA], om = (T)d->scal[SC_OMEGA];
        for (int a = 0; a < bs; ++a) {
            int64_t k = pn * bs + a;
            vp<T>(d->kx)[k] += al * vp<T>(d->kph)[k] + om * vp<T>(d->ksh)[k];
            T r = vp<T>(d->ks)[k] - om * vp<T>(d->kt)[k];
            vp<T>(d->kr)[k] = r;
            v[0] += (double)vp<T>(d->kh)[k] * (double)r;
            v[1] += (double)r * (double)r;
        }
    }
    block_partials<2>(d, lb, v);
}

// scalar updates, one block per problem; stage:
//   0 after init: rho = (r,r), tol2, alpha = omega = 1, beta = 0
//   1 after v = J ph: alpha = rho / (rhat, v)
//   2 after t = J sh: omega = (t, s) / (t, t)
//   3 after x, r: beta, rho, convergence
__global__ void k_bicg_scalars(Batch B, int stage, double rtol, int maxit) {
    const int q = blockIdx.x;
    const Dev* d = B.d[q];
    if (stage != 0 && krylov_done(d)) return;
    __shared__ double sh[2][TPB];
    const int64_t nblk = (d->Nnode + TPB - 1) / TPB;
    double a = 0.0, b2 = 0.0;
    for (int64_t i = threadIdx.x; i < nblk; i += TPB) {
        a += d->partial[i * 4 + 0];
        b2 += d->partial[i * 4 + 1];
    }
    sh[0][threadIdx.x] = a;
    sh[1][threadIdx.x] = b2;
    __syncthreads();
    for (int off = TPB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + off];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    double* sc = d->scal;
    double s0 = sh[0][0], s1 = sh[1][0];
    if (stage == 0) {
        sc[SC_RHO] = s0;
        sc[SC_RR] = s0;
        sc[SC_TOL2] = rtol * rtol * s0;
        sc[SC_ALPHA] = 1.0;
        sc[SC_OMEGA] = 1.0;
        sc[SC_BETA] = 0.0;
        sc[SC_ITER] = 0.0;
        sc[SC_BREAK] = 0.0;
        sc[SC_DONE] = (s0 == 0.0 || maxit <= 0) ? 1.0 : 0.0;
    } else if (stage == 1) {
        sc[SC_RV] = s0;
        if (s0 == 0.0 || !isfinite(s0)) { sc[SC_BREAK] = 1.0; sc[SC_DONE] = 1.0; return; }
        sc[SC_ALPHA] = sc[SC_RHO] / s0;
    } else if (stage == 2) {
        sc[SC_TS] = s0;
        sc[SC_TT] = s1;
        if (s1 == 0.0 || !isfinite(s1)) {
            // t = 0: s is already the exact residual of x + alpha ph; take omega = 0
            sc[SC_OMEGA] = 0.0;
            return;
        }
        sc[SC_OMEGA] = s0 / s1;
    } else {
        double rho_new = s0;
        sc[SC_RR] = s1;
        sc[SC_ITER] += 1.0;
        bool conv = s1 <= sc[SC_TOL2];
        bool brk = (rho_new == 0.0 || sc[SC_OMEGA] == 0.0 || !isfinite(s1));
        if (!conv && brk) sc[SC_BREAK] = 1.0;
        if (conv || brk || sc[SC_ITER] >= (double)maxit) {
            sc[SC_DONE] = 1.0;
            return;
        }
        sc[SC_BETA] = (rho_new / sc[SC_RHO]) * (sc[SC_ALPHA] / sc[SC_OMEGA]);
        sc[SC_RHO] = rho_new;
    }
}

// X += x (Newton update, FP64)
template <typename T>
__global__ void __launch_bounds__(TPB) k_newton_update(Batch B) {
    PROB_PROLOGUE
    if (tid >= d->Nnode) return;
    const int64_t pn = node_pad<T>(d, tid);
    const int bs = d->b;
    for (int a = 0; a < bs; ++a) {
        int64_t k = pn * bs + a;
        if (d->dfree[k]) d->X[k] += (double)vp<T>(d->kx)[k];
    }
}

// ---------------------------------------------------------------------------------------------
// multigrid
// ---------------------------------------------------------------------------------------------
// Operator entry (row, stencil s, a, c) of family F (0: A, block DIM; 1: S, block 1) on level l.
// Level 0 reads the Jacobian; family S adds the fixed-stress diagonal.
template <typename T>
struct Op {
    const T* base;
    int64_t nrow;
    int BJ;      // block size of the storage
    int a0;      // first storage row/col of the family
    __device__ __forceinline__ double at(int s, int a, int c, int64_t row) const {
        return (double)base[((int64_t)(s * BJ + a + a0) * BJ + c + a0) * nrow + row];
    }
};

template <typename T>
__device__ __forceinline__ Op<T> op_of(const Dev* d, int fam, int l) {
    Op<T> o;
    if (l == 0) {
        o.base = (const T*)d->J;
        o.nrow = d->Nnode;
        o.BJ = d->b;
        o.a0 = fam == 0 ? 0 : d->dim;
    } else {
        o.base = (const T*)(fam == 0 ? d->lev[l].A : d->lev[l].Sm);
        o.nrow = d->lev[l].nrow;
        o.BJ = fam == 0 ? d->dim : 1;
        o.a0 = 0;
    }
    return o;
}

// fixed-stress diagonal term of S on level 0 (zero on non-free pressure dofs)
__device__ __forceinline__ double fs_term(const Dev* d, int64_t pn) {
    return d->dfree[pn * d->b + d->dim] ? d->ct / d->Kfs * d->Mp[pn] : 0.0;
}

__device__ __forceinline__ double mask0(const Dev* d, int fam, int64_t pn, int comp) {
    return d->dfree[pn * d->b + (fam == 0 ? comp : d->dim)] ? 1.0 : 0.0;
}

// 1D prolongation weight of fine node i from coarse node I (n_f fine nodes on the axis)
__device__ __forceinline__ double pw1(int i, int I, int nf) {
    if ((i & 1) == 0) return I == (i >> 1) ? 1.0 : 0.0;
    int lo = (i - 1) >> 1, hi = lo + 1;
    int phi = min(2 * hi, nf - 1);
    if (phi == i) return I == hi ? 1.0 : 0.0;
    return (I == lo || I == hi) ? 0.5 : 0.0;
}

template <int BB>
__device__ __forceinline__ bool invert_small(const double* A, double* Ai) {
    if (BB == 1) {
        if (A[0] == 0.0 || !isfinite(A[0])) { Ai[0] = 1.0; return false; }
        Ai[0] = 1.0 / A[0];
        return true;
    }
    double dt = BB == 2 ? det<2>(A) : det<3>(A);
    if (dt == 0.0 || !isfinite(dt)) {
        for (int i = 0; i < BB * BB; ++i) Ai[i] = (i % (BB + 1) == 0) ? 1.0 : 0.0;
        return false;
    }
    if (BB == 2) inverse<2>(A, Ai);
    else inverse<3>(A, Ai);
    return true;
}

// inverse diagonal blocks of level l, family fam (block BB)
template <int BB, typename T>
__global__ void __launch_bounds__(TPB) k_mg_dinv(Batch B, int fam, int l) {
    PROB_PROLOGUE
    if (l >= d->nlev) return;
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

// Galerkin coarse operator of level l+1 from level l: thread per (coarse row, stencil entry)
template <int BB, typename T>
__global__ void __launch_bounds__(TPB) k_mg_rap(Batch B, int fam, int l) {
    PROB_PROLOGUE
    if (l + 1 >= d->nlev) return;
    const MgLevel& F = d->lev[l];
    const MgLevel& C = d->lev[l + 1];
    if (tid >= C.nrow) return;
    const int s = blockIdx.y;
    const int dim = d->dim, R = d->R, SW = 2 * R + 1;
    int I[3], Jc[3], off[3] = {s % SW - R, (s / SW) % SW - R, dim == 3 ? s / (SW * SW) - R : 0};
    real_coords(tid, C.n, dim, I);
    bool valid = true;
    for (int a = 0; a < dim; ++a) {
        Jc[a] = I[a] + off[a];
        if (Jc[a] < 0 || Jc[a] >= C.n[a]) valid = false;
    }
    double blk[BB * BB];
    for (int k = 0; k < BB * BB; ++k) blk[k] = 0.0;
    if (valid) {
        Op<T> o = op_of<T>(d, fam, l);
        const int nI = dim == 3 ? 27 : 9;
        for (int ii = 0; ii < nI; ++ii) {
            int fi[3] = {2 * I[0] - 1 + ii % 3, 2 * I[1] - 1 + (ii / 3) % 3, dim == 3 ? 2 * I[2] - 1 + ii / 9 : 0};
            double wi = 1.0;
            for (int a = 0; a < dim; ++a) {
                if (fi[a] < 0 || fi[a] >= F.n[a]) { wi = 0.0; break; }
                wi *= pw1(fi[a], I[a], F.n[a]);
            }
            if (wi == 0.0) continue;
            int64_t frow = fi[0] + (int64_t)F.n[0] * (fi[1] + (int64_t)F.n[1] * fi[2]);
            int64_t fpn = padded(fi, F.np, R, dim);
            for (int jj = 0; jj < nI; ++jj) {
                int fj[3] = {2 * Jc[0] - 1 + jj % 3, 2 * Jc[1] - 1 + (jj / 3) % 3, dim == 3 ? 2 * Jc[2] - 1 + jj / 9 : 0};
                double wj = 1.0;
                int fs = 0, mul = 1;
                for (int a = 0; a < dim; ++a) {
                    if (fj[a] < 0 || fj[a] >= F.n[a]) { wj = 0.0; break; }
                    int dd = fj[a] - fi[a];
                    if (dd < -R || dd > R) { wj = 0.0; break; }
                    wj *= pw1(fj[a], Jc[a], F.n[a]);
                    fs += (dd + R) * mul;
                    mul *= SW;
                }
                if (wj == 0.0) continue;
                int64_t fpnj = padded(fj, F.np, R, dim);
                double w = wi * wj;
                for (int a = 0; a < BB; ++a) {
                    double mi = l == 0 ? mask0(d, fam, fpn, a) : 1.0;
                    if (mi == 0.0) continue;
                    for (int c = 0; c < BB; ++c) {
                        double mj = l == 0 ? mask0(d, fam, fpnj, c) : 1.0;
                        if (mj == 0.0) continue;
                        double v = o.at(fs, a, c, frow);
                        if (fam == 1 && l == 0 && fs == (d->S - 1) / 2) v += fs_term(d, fpn);
                        blk[a * BB + c] += w * v;
                    }
                }
            }
        }
        if (s == (d->S - 1) / 2)
            for (int a = 0; a < BB; ++a)
                if (blk[a * BB + a] == 0.0) blk[a * BB + a] = 1.0;
    }
    T* out = (T*)(fam == 0 ? C.A : C.Sm);
    for (int a = 0; a < BB; ++a)
        for (int c = 0; c < BB; ++c) out[((int64_t)(s * BB + a) * BB + c) * C.nrow + tid] = (T)blk[a * BB + c];
}

// dense inverse of the coarsest operator: Gauss-Jordan with partial pivoting in FP64, one block
// per problem, on the workspace matrix cwork (n <= CMAX)
template <int BB, typename T>
__global__ void __launch_bounds__(1024) k_mg_coarse_setup(Batch B, int fam) {
    const int q = blockIdx.x;
    const Dev* d = B.d[q];
    const int l = d->nlev - 1;
    const MgLevel& L = d->lev[l];
    const int dim = d->dim, R = d->R;
    const int n = (int)(L.nrow * BB);
    if (n > CMAX) return;
    double* M = d->cwork;
    __shared__ int piv;
    __shared__ int perm[CMAX];
    Op<T> o = op_of<T>(d, fam, l);
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) M[e] = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) perm[i] = i;
    __syncthreads();
    for (int e = threadIdx.x; e < L.nrow * d->S; e += blockDim.x) {
        int64_t row = e % L.nrow;
        int s = (int)(e / L.nrow);
        int c0[3], c1[3];
        real_coords(row, L.n, dim, c0);
        int SW = 2 * R + 1;
        int off[3] = {s % SW - R, (s / SW) % SW - R, dim == 3 ? s / (SW * SW) - R : 0};
        bool ok = true;
        for (int a = 0; a < dim; ++a) {
            c1[a] = c0[a] + off[a];
            if (c1[a] < 0 || c1[a] >= L.n[a]) ok = false;
        }
        if (dim == 2) c1[2] = 0;
        if (!ok) continue;
        int64_t col = c1[0] + (int64_t)L.n[0] * (c1[1] + (int64_t)L.n[1] * c1[2]);
        for (int a = 0; a < BB; ++a)
            for (int c = 0; c < BB; ++c) {
                double v = o.at(s, a, c, row);
                if (fam == 1 && l == 0 && s == (d->S - 1) / 2) v += fs_term(d, padded(c0, L.np, R, dim));
                M[(row * BB + a) * n + col * BB + c] = v;
            }
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (threadIdx.x == 0) {
            int best = k;
            double bv = fabs(M[k * n + k]);
            for (int r = k + 1; r < n; ++r)
                if (fabs(M[r * n + k]) > bv) { bv = fabs(M[r * n + k]); best = r; }
            piv = best;
        }
        __syncthreads();
        const int pr = piv;
        if (pr != k) {
            for (int c = threadIdx.x; c < n; c += blockDim.x) {
                double t = M[k * n + c]; M[k * n + c] = M[pr * n + c]; M[pr * n + c] = t;
            }
            if (threadIdx.x == 0) { int t = perm[k]; perm[k] = perm[pr]; perm[pr] = t; }
        }
        __syncthreads();
        double pv = M[k * n + k];
        if (pv == 0.0 || !isfinite(pv)) pv = 1.0;
        __syncthreads();
        for (int c = threadIdx.x; c < n; c += blockDim.x)
            if (c != k) M[k * n + c] /= pv;
        __syncthreads();
        if (threadIdx.x == 0) M[k * n + k] = 1.0 / pv;
        __syncthreads();
        for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
            int r = e / n, c = e % n;
            if (r == k || c == k) continue;
            M[r * n + c] -= M[r * n + k] * M[k * n + c];
        }
        __syncthreads();
        for (int r = threadIdx.x; r < n; r += blockDim.x)
            if (r != k) M[r * n + k] = -M[r * n + k] * M[k * n + k];
        __syncthreads();
    }
    // the row swaps of the factorization permute the columns of the inverse
    T* out = (T*)(fam == 0 ? d->cinvA : d->cinvS);
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        int r = e / n, c = e % n;
        out[(int64_t)r * n + perm[c]] = (T)M[r * n + c];
    }
}

// Symbolic vector reference resolved per problem inside the kernels, so that one launch serves
// every problem of a batch: kinds 0..8 are the Krylov vectors (x r rhat p v s t ph sh, block b,
// component offset `off`), 9 is the rhs of the A cycle on level 0 (block dim), 10/11/12 are the
// level solution / residual / right-hand side of the family being cycled (block BB).
struct VRef {
    int kind;
    int off;
};
enum { VK_BT = 9, VK_LX = 10, VK_LR = 11, VK_LB = 12 };

template <typename T>
struct View {
    T* p;
    int stride, off;
    __device__ __forceinline__ T& at(int64_t pn, int c) const { return p[pn * stride + off + c]; }
};

template <typename T>
__device__ __forceinline__ View<T> resolve(const Dev* d, VRef v, int fam, int l, int BB) {
    View<T> o;
    o.off = v.off;
    if (v.kind < 9) {
        void* const vecs[9] = {d->kx, d->kr, d->kh, d->kp, d->kv, d->ks, d->kt, d->kph, d->ksh};
        o.p = (T*)vecs[v.kind];
        o.stride = d->b;
    } else if (v.kind == VK_BT) {
        o.p = (T*)d->kbt;
        o.stride = d->dim;
    } else {
        const MgLevel& L = d->lev[l];
        void* p;
        if (v.kind == VK_LX) p = fam == 0 ? L.xa : L.xs;
        else if (v.kind == VK_LR) p = fam == 0 ? L.ra : L.rs;
        else p = fam == 0 ? L.ba : L.bsv;
        o.p = (T*)p;
        o.stride = BB;
    }
    return o;
}

// x = omega Dinv rhs  (levels below the coarsest of the problem)
template <int BB, typename T>
__global__ void __launch_bounds__(TPB) k_mg_smooth0(Batch B, int fam, int l, VRef rv, VRef xv) {
    PROB_PROLOGUE
    if (krylov_done(d) || l >= d->nlev - 1) return;
    const MgLevel& L = d->lev[l];
    if (tid >= L.nrow) return;
    View<T> rhs = resolve<T>(d, rv, fam, l, BB), x = resolve<T>(d, xv, fam, l, BB);
    int c[3];
    real_coords(tid, L.n, d->dim, c);
    int64_t pn = padded(c, L.np, d->R, d->dim);
    const T* Di = (const T*)(fam == 0 ? L.Ad : L.Sd);
    double r[BB];
    for (int a = 0; a < BB; ++a) r[a] = (double)rhs.at(pn, a);
    for (int a = 0; a < BB; ++a) {
        double t = 0.0;
        for (int cc = 0; cc < BB; ++cc) t += (double)Di[(int64_t)(a * BB + cc) * L.nrow + tid] * r[cc];
        x.at(pn, a) = (T)(d->omega * t);
    }
}

// r = rhs - A x
template <int BB, typename T>
__global__ void __launch_bounds__(TPB) k_mg_resid(Batch B, int fam, int l, VRef rv, VRef xv, VRef resv) {
    PROB_PROLOGUE
    if (krylov_done(d) || l >= d->nlev - 1) return;
    const MgLevel& L = d->lev[l];
    if (tid >= L.nrow) return;
    View<T> rhs = resolve<T>(d, rv, fam, l, BB), x = resolve<T>(d, xv, fam, l, BB), r = resolve<T>(d, resv, fam, l, BB);
    const int dim = d->dim, R = d->R;
    int c[3];
    real_coords(tid, L.n, dim, c);
    int64_t pn = padded(c, L.np, R, dim);
    Op<T> o = op_of<T>(d, fam, l);
    double acc[BB];
    for (int a = 0; a < BB; ++a) acc[a] = (double)rhs.at(pn, a);
    for (int s = 0; s < d->S; ++s) {
        int64_t pk = pn + stencil_offset(s, R, dim, L.np);
        for (int cc = 0; cc < BB; ++cc) {
            double xv2 = (double)x.at(pk, cc);
            for (int a = 0; a < BB; ++a) acc[a] -= o.at(s, a, cc, tid) * xv2;
        }
    }
    if (fam == 1 && l == 0) acc[0] -= fs_term(d, pn) * (double)x.at(pn, 0);
    for (int a = 0; a < BB; ++a) r.at(pn, a) = (T)acc[a];
}

// x += omega Dinv r
template <int BB, typename T>
__global__ void __launch_bounds__(TPB) k_mg_update(Batch B, int fam, int l, VRef xv, VRef resv) {
    PROB_PROLOGUE
    if (krylov_done(d) || l >= d->nlev - 1) return;
    const MgLevel& L = d->lev[l];
    if (tid >= L.nrow) return;
    View<T> x = resolve<T>(d, xv, fam, l, BB), r = resolve<T>(d, resv, fam, l, BB);
    int c[3];
    real_coords(tid, L.n, d->dim, c);
    int64_t pn = padded(c, L.np, d->R, d->dim);
    const T* Di = (const T*)(fam == 0 ? L.Ad : L.Sd);
    double rr[BB];
    for (int a = 0; a < BB; ++a) rr[a] = (double)r.at(pn, a);
    for (int a = 0; a < BB; ++a) {
        double t = 0.0;
        for (int cc = 0; cc < BB; ++cc) t += (double)Di[(int64_t)(a * BB + cc) * L.nrow + tid] * rr[cc];
        x.at(pn, a) = (T)((double)x.at(pn, a) + d->omega * t);
    }
}

// coarse rhs = P^T r (level-0 fine dofs masked)
template <int BB, typename T>
__global__ void __launch_bounds__(TPB) k_mg_restrict(Batch B, int fam, int l, VRef rv, VRef bv) {
    PROB_PROLOGUE
    if (krylov_done(d) || l + 1 >= d->nlev) return;
    const MgLevel& F = d->lev[l];
    const MgLevel& C = d->lev[l + 1];
    if (tid >= C.nrow) return;
    View<T> r = resolve<T>(d, rv, fam, l, BB), bc = resolve<T>(d, bv, fam, l + 1, BB);
    const int dim = d->dim, R = d->R;
    int I[3];
    real_coords(tid, C.n, dim, I);
    double acc[BB];
    for (int a = 0; a < BB; ++a) acc[a] = 0.0;
    const int nI = dim == 3 ? 27 : 9;
    for (int ii = 0; ii < nI; ++ii) {
        int fi[3] = {2 * I[0] - 1 + ii % 3, 2 * I[1] - 1 + (ii / 3) % 3, dim == 3 ? 2 * I[2] - 1 + ii / 9 : 0};
        double w = 1.0;
        for (int a = 0; a < dim; ++a) {
            if (fi[a] < 0 || fi[a] >= F.n[a]) { w = 0.0; break; }
            w *= pw1(fi[a], I[a], F.n[a]);
        }
        if (w == 0.0) continue;
        int64_t fpn = padded(fi, F.np, R, dim);
        for (int a = 0; a < BB; ++a) {
            double m = l == 0 ? mask0(d, fam, fpn, a) : 1.0;
            acc[a] += w * m * (double)r.at(fpn, a);
        }
    }
    int64_t cpn = padded(I, C.np, R, dim);
    for (int a = 0; a < BB; ++a) bc.at(cpn, a) = (T)acc[a];
}

// x += P xc (level-0 fine dofs masked)
template <int BB, typename T>
__global__ void __launch_bounds__(TPB) k_mg_prolong(Batch B, int fam, int l, VRef xcv, VRef xv) {
    PROB_PROLOGUE
    if (krylov_done(d) || l + 1 >= d->nlev) return;
    const MgLevel& F = d->lev[l];
    const MgLevel& C = d->lev[l + 1];
    if (tid >= F.nrow) return;
    View<T> xc = resolve<T>(d, xcv, fam, l + 1, BB), x = resolve<T>(d, xv, fam, l, BB);
    const int dim = d->dim, R = d->R;
    int fi[3];
    real_coords(tid, F.n, dim, fi);
    int64_t fpn = padded(fi, F.np, R, dim);
    double acc[BB];
    for (int a = 0; a < BB; ++a) acc[a] = 0.0;
    const int nI = dim == 3 ? 8 : 4;
    for (int jj = 0; jj < nI; ++jj) {
        int I[3] = {0, 0, 0};
        double w = 1.0;
        for (int a = 0; a < dim; ++a) {
            int lo = fi[a] >> 1;
            I[a] = lo + ((jj >> a) & 1);
            if (I[a] >= C.n[a]) { w = 0.0; break; }
            w *= pw1(fi[a], I[a], F.n[a]);
        }
        if (w == 0.0) continue;
        int64_t cpn = padded(I, C.np, R, dim);
        for (int a = 0; a < BB; ++a) acc[a] += w * (double)xc.at(cpn, a);
    }
    for (int a = 0; a < BB; ++a) {
        double m = l == 0 ? mask0(d, fam, fpn, a) : 1.0;
        x.at(fpn, a) = (T)((double)x.at(fpn, a) + m * acc[a]);
    }
}

// coarsest level of each problem: x = Cinv rhs (one block per problem)
template <int BB, typename T>
__global__ void __launch_bounds__(TPB) k_mg_coarse(Batch B, int fam, int l, VRef rv, VRef xv) {
    const int q = blockIdx.x;
    const Dev* d = B.d[q];
    if (krylov_done(d) || l != d->nlev - 1) return;
    const MgLevel& L = d->lev[l];
    View<T> rhs = resolve<T>(d, rv, fam, l, BB), x = resolve<T>(d, xv, fam, l, BB);
    const int n = (int)(L.nrow * BB);
    if (n > CMAX) return;   // excluded when the problem is created
    const T* Ci = (const T*)(fam == 0 ? d->cinvA : d->cinvS);
    __shared__ double rvv[CMAX];
    const int dim = d->dim, R = d->R;
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        int c[3];
        real_coords(e / BB, L.n, dim, c);
        rvv[e] = (double)rhs.at(padded(c, L.np, R, dim), e % BB);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
        double t = 0.0;
        for (int k = 0; k < n; ++k) t += (double)Ci[(int64_t)e * n + k] * rvv[k];
        int c[3];
        real_coords(e / BB, L.n, dim, c);
        x.at(padded(c, L.np, R, dim), e % BB) = (T)t;
    }
}

// t_u = y_u - B1 z_p on level 0 (B1 = displacement rows, pressure columns of J)
template <int DIM, typename T>
__global__ void __launch_bounds__(TPB) k_b1(Batch B, VRef yv, VRef zv) {
    PROB_PROLOGUE
    if (krylov_done(d) || tid >= d->Nnode) return;
    View<T> y = resolve<T>(d, yv, 0, 0, DIM), z = resolve<T>(d, zv, 0, 0, 1), t = resolve<T>(d, VRef{VK_BT, 0}, 0, 0, DIM);
    const int R = d->R, bs = d->b;
    int c[3];
    real_coords(tid, d->nn, DIM, c);
    int64_t pn = padded(c, d->np1, R, DIM);
    const T* J = (const T*)d->J;
    const int64_t Nn = d->Nnode;
    double acc[DIM];
    for (int a = 0; a < DIM; ++a) acc[a] = (double)y.at(pn, a);
    for (int s = 0; s < d->S; ++s) {
        int64_t pk = pn + stencil_offset(s, R, DIM, d->np1);
        double zp = (double)z.at(pk, 0);
        for (int a = 0; a < DIM; ++a) acc[a] -= (double)J[((int64_t)(s * bs + a) * bs + DIM) * Nn + tid] * zp;
    }
    for (int a = 0; a < DIM; ++a) t.at(pn, a) = (T)acc[a];
}

// ---------------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------------
static std::vector<int64_t> level_rows(const std::vector<const Dev*>& hc, int l) {
    std::vector<int64_t> v;
    for (auto* h : hc) v.push_back(l < h->nlev ? h->lev[l].nrow : 1);
    return v;
}

static int max_levels(const std::vector<const Dev*>& hc) {
    int L = 0;
    for (auto* h : hc) L = std::max(L, h->nlev);
    return L;
}

template <int DIM, typename T>
static void precond_setup_t(const Group& g, const std::vector<const Dev*>& hc, hipStream_t st) {
    const int Lmax = max_levels(hc);
    for (int l = 0; l < Lmax; ++l) {
        Batch Bl = make_batch(g.ddev, level_rows(hc, l), TPB);
        hipLaunchKernelGGL((k_mg_dinv<DIM, T>), dim3(Bl.pfx[Bl.n]), dim3(TPB), 0, st, Bl, 0, l);
        hipLaunchKernelGGL((k_mg_dinv<1, T>), dim3(Bl.pfx[Bl.n]), dim3(TPB), 0, st, Bl, 1, l);
        if (l + 1 < Lmax) {
            Batch Bc = make_batch(g.ddev, level_rows(hc, l + 1), TPB);
            PPM_TIMED(KT_RAP, st, hipLaunchKernelGGL((k_mg_rap<DIM, T>), dim3(Bc.pfx[Bc.n], g.S), dim3(TPB), 0, st, Bc, 0, l));
            hipLaunchKernelGGL((k_mg_rap<1, T>), dim3(Bc.pfx[Bc.n], g.S), dim3(TPB), 0, st, Bc, 1, l);
        }
    }
    Batch B1 = make_batch_one_block(g.ddev);
    hipLaunchKernelGGL((k_mg_coarse_setup<DIM, T>), dim3(B1.n), dim3(1024), 0, st, B1, 0);
    hipLaunchKernelGGL((k_mg_coarse_setup<1, T>), dim3(B1.n), dim3(1024), 0, st, B1, 1);
}

void launch_precond_setup(const Group& g, const std::vector<const Dev*>& hc, hipStream_t st) {
    if (g.dim == 2) {
        if (g.mixed) precond_setup_t<2, float>(g, hc, st);
        else precond_setup_t<2, double>(g, hc, st);
    } else {
        if (g.mixed) precond_setup_t<3, float>(g, hc, st);
        else precond_setup_t<3, double>(g, hc, st);
    }
}

// One batched V-cycle of family fam (block BB): level-0 right-hand side rhs0 and solution out0
// are Krylov-vector references; deeper levels use each problem's own level vectors.
template <int BB, typename T>
static void vcycle(const Group& g, const std::vector<const Dev*>& hc, int fam, VRef rhs0, VRef out0, int nsm,
                   hipStream_t st) {
    const int Lmax = max_levels(hc);
    Batch B1 = make_batch_one_block(g.ddev);
    const VRef LX{VK_LX, 0}, LR{VK_LR, 0}, LB{VK_LB, 0};
    for (int l = 0; l < Lmax; ++l) {
        const VRef rhs = l == 0 ? rhs0 : LB, x = l == 0 ? out0 : LX;
        hipLaunchKernelGGL((k_mg_coarse<BB, T>), dim3(B1.n), dim3(TPB), 0, st, B1, fam, l, rhs, x);
        if (l + 1 >= Lmax) break;
        Batch Bl = make_batch(g.ddev, level_rows(hc, l), TPB);
        const dim3 gl(Bl.pfx[Bl.n]);
        hipLaunchKernelGGL((k_mg_smooth0<BB, T>), gl, dim3(TPB), 0, st, Bl, fam, l, rhs, x);
        for (int k = 1; k < nsm; ++k) {
            PPM_TIMED((l == 0 ? KT_MG0_RESID : -1), st, hipLaunchKernelGGL((k_mg_resid<BB, T>), gl, dim3(TPB), 0, st, Bl, fam, l, rhs, x, LR));
            hipLaunchKernelGGL((k_mg_update<BB, T>), gl, dim3(TPB), 0, st, Bl, fam, l, x, LR);
        }
        PPM_TIMED((l == 0 ? KT_MG0_RESID : -1), st, hipLaunchKernelGGL((k_mg_resid<BB, T>), gl, dim3(TPB), 0, st, Bl, fam, l, rhs, x, LR));
        Batch Bc = make_batch(g.ddev, level_rows(hc, l + 1), TPB);
        hipLaunchKernelGGL((k_mg_restrict<BB, T>), dim3(Bc.pfx[Bc.n]), dim3(TPB), 0, st, Bc, fam, l, LR, LB);
    }
    for (int l = Lmax - 2; l >= 0; --l) {
        const VRef rhs = l == 0 ? rhs0 : LB, x = l == 0 ? out0 : LX;
        Batch Bl = make_batch(g.ddev, level_rows(hc, l), TPB);
        const dim3 gl(Bl.pfx[Bl.n]);
        hipLaunchKernelGGL((k_mg_prolong<BB, T>), gl, dim3(TPB), 0, st, Bl, fam, l, LX, x);
        for (int k = 0; k < nsm; ++k) {
            PPM_TIMED((l == 0 ? KT_MG0_RESID : -1), st, hipLaunchKernelGGL((k_mg_resid<BB, T>), gl, dim3(TPB), 0, st, Bl, fam, l, rhs, x, LR));
            hipLaunchKernelGGL((k_mg_update<BB, T>), gl, dim3(TPB), 0, st, Bl, fam, l, x, LR);
        }
    }
}

// z = P^-1 y on Krylov vectors iy -> iz: Schur block first, then A
template <int DIM, typename T>
static void precond_apply(const Group& g, const std::vector<const Dev*>& hc, int iy, int iz, hipStream_t st) {
    const int nsm = hc[0]->mg_nsm;
    vcycle<1, T>(g, hc, 1, VRef{iy, DIM}, VRef{iz, DIM}, nsm, st);
    Batch Bn = make_batch(g.ddev, g.nnode, TPB);
    hipLaunchKernelGGL((k_b1<DIM, T>), dim3(Bn.pfx[Bn.n]), dim3(TPB), 0, st, Bn, VRef{iy, 0}, VRef{iz, DIM});
    vcycle<DIM, T>(g, hc, 0, VRef{VK_BT, 0}, VRef{iz, 0}, nsm, st);
}

template <int DIM, int R, typename T>
static void krylov_iters_t(const Group& g, const std::vector<const Dev*>& hc, int iters, double rtol, int maxit,
                           hipStream_t st) {
    Batch Bn = make_batch(g.ddev, g.nnode, TPB);
    Batch B1 = make_batch_one_block(g.ddev);
    const dim3 gN(Bn.pfx[Bn.n]), tb(TPB);
    // vector ids: 0 x, 1 r, 2 rhat, 3 p, 4 v, 5 s, 6 t, 7 ph, 8 sh
    for (int it = 0; it < iters; ++it) {
        hipLaunchKernelGGL(k_bicg_p<T>, gN, tb, 0, st, Bn);
        precond_apply<DIM, T>(g, hc, 3, 7, st);
        PPM_TIMED(KT_SPMV, st, hipLaunchKernelGGL((k_spmv<DIM, R, T>), gN, tb, 0, st, Bn, 7, 4, 2, 1, 1));
        hipLaunchKernelGGL(k_bicg_scalars, dim3(B1.n), tb, 0, st, B1, 1, rtol, maxit);
        hipLaunchKernelGGL(k_bicg_s<T>, gN, tb, 0, st, Bn);
        precond_apply<DIM, T>(g, hc, 5, 8, st);
        PPM_TIMED(KT_SPMV, st, hipLaunchKernelGGL((k_spmv<DIM, R, T>), gN, tb, 0, st, Bn, 8, 6, 5, 2, 1));
        hipLaunchKernelGGL(k_bicg_scalars, dim3(B1.n), tb, 0, st, B1, 2, rtol, maxit);
        hipLaunchKernelGGL(k_bicg_xr<T>, gN, tb, 0, st, Bn);
        hipLaunchKernelGGL(k_bicg_scalars, dim3(B1.n), tb, 0, st, B1, 3, rtol, maxit);
    }
}

void launch_krylov_init(const Group& g, double rtol, int maxit, hipStream_t st) {
    Batch Bn = make_batch(g.ddev, g.nnode, TPB);
    Batch B1 = make_batch_one_block(g.ddev);
    if (g.mixed) hipLaunchKernelGGL(k_bicg_init<float>, dim3(Bn.pfx[Bn.n]), dim3(TPB), 0, st, Bn);
    else hipLaunchKernelGGL(k_bicg_init<double>, dim3(Bn.pfx[Bn.n]), dim3(TPB), 0, st, Bn);
    hipLaunchKernelGGL(k_bicg_scalars, dim3(B1.n), dim3(TPB), 0, st, B1, 0, rtol, maxit);
}

void launch_krylov_iters(const Group& g, const std::vector<const Dev*>& hc, int iters, double rtol, int maxit,
                         hipStream_t st) {
    int R = g.shape ? 2 : 1;
    if (g.dim == 2 && R == 1) {
        if (g.mixed) krylov_iters_t<2, 1, float>(g, hc, iters, rtol, maxit, st);
        else krylov_iters_t<2, 1, double>(g, hc, iters, rtol, maxit, st);
    } else if (g.dim == 2) {
        if (g.mixed) krylov_iters_t<2, 2, float>(g, hc, iters, rtol, maxit, st);
        else krylov_iters_t<2, 2, double>(g, hc, iters, rtol, maxit, st);
    } else {
        if (g.mixed) krylov_iters_t<3, 1, float>(g, hc, iters, rtol, maxit, st);
        else krylov_iters_t<3, 1, double>(g, hc, iters, rtol, maxit, st);
    }
}

void launch_newton_update(const Group& g, hipStream_t st) {
    Batch Bn = make_batch(g.ddev, g.nnode, TPB);
    if (g.mixed) hipLaunchKernelGGL(k_newton_update<float>, dim3(Bn.pfx[Bn.n]), dim3(TPB), 0, st, Bn);
    else hipLaunchKernelGGL(k_newton_update<double>, dim3(Bn.pfx[Bn.n]), dim3(TPB), 0, st, Bn);
}

// ---------------------------------------------------------------------------------------------
// inspection helpers: natural-order <-> padded conversions, y = J v
// ---------------------------------------------------------------------------------------------
template <typename T>
__global__ void k_nat_to_pad(Batch B, const double* __restrict__ v, int which) {
    PROB_PROLOGUE
    if (tid >= d->Nnode) return;
    const int64_t pn = node_pad<T>(d, tid);
    const int bs = d->b;
    for (int a = 0; a < bs; ++a) {
        double x = v[tid * bs + a];
        if (which == 0) vp<T>(d->kp)[pn * bs + a] = (T)x;
    }
}

template <typename T>
__global__ void k_pad_to_nat(Batch B, double* __restrict__ out, int which) {
    PROB_PROLOGUE
    if (tid >= d->Nnode) return;
    const int64_t pn = node_pad<T>(d, tid);
    const int bs = d->b;
    for (int a = 0; a < bs; ++a) {
        int64_t k = pn * bs + a;
        double v;
        if (which == 0) v = (double)vp<T>(d->kv)[k];
        else if (which == 1) v = d->Rv[k];
        else if (which == 2) v = (double)d->dfree[k];
        else v = 0.0;
        out[tid * bs + a] = v;
    }
}

__global__ void k_nodal_scalar_out(Batch B, double* __restrict__ out, int field) {
    PROB_PROLOGUE
    if (tid >= d->Nnode) return;
    int c[3];
    real_coords(tid, d->nn, d->dim, c);
    int64_t pn = padded(c, d->np1, d->R, d->dim);
    out[tid] = field == 0 ? d->M[pn] : d->Pn[pn];
}

__global__ void k_set_state(Batch B, const double* __restrict__ U, const double* __restrict__ P) {
    PROB_PROLOGUE
    if (tid >= d->Nnode) return;
    int c[3];
    real_coords(tid, d->nn, d->dim, c);
    int64_t pn = padded(c, d->np1, d->R, d->dim);
    const int D = d->dim, bs = d->b;
    for (int a = 0; a < D; ++a) d->X[pn * bs + a] = U[tid * D + a];
    d->X[pn * bs + D] = P[tid];
}

void launch_apply_jacobian(const Dev* dd, const Dev* hd, const double* v_nat, double* y_nat, hipStream_t st) {
    Batch Bn = make_batch({dd}, {hd->Nnode}, TPB);
    const dim3 gN(Bn.pfx[1]), tb(TPB);
    int R = hd->R;
    if (hd->mixed) {
        hipLaunchKernelGGL(k_nat_to_pad<float>, gN, tb, 0, st, Bn, v_nat, 0);
        if (hd->dim == 2 && R == 1) hipLaunchKernelGGL((k_spmv<2, 1, float>), gN, tb, 0, st, Bn, 3, 4, 0, 0, 0);
        else if (hd->dim == 2) hipLaunchKernelGGL((k_spmv<2, 2, float>), gN, tb, 0, st, Bn, 3, 4, 0, 0, 0);
        else hipLaunchKernelGGL((k_spmv<3, 1, float>), gN, tb, 0, st, Bn, 3, 4, 0, 0, 0);
        hipLaunchKernelGGL(k_pad_to_nat<float>, gN, tb, 0, st, Bn, y_nat, 0);
    } else {
        hipLaunchKernelGGL(k_nat_to_pad<double>, gN, tb, 0, st, Bn, v_nat, 0);
        if (hd->dim == 2 && R == 1) hipLaunchKernelGGL((k_spmv<2, 1, double>), gN, tb, 0, st, Bn, 3, 4, 0, 0, 0);
        else if (hd->dim == 2) hipLaunchKernelGGL((k_spmv<2, 2, double>), gN, tb, 0, st, Bn, 3, 4, 0, 0, 0);
        else hipLaunchKernelGGL((k_spmv<3, 1, double>), gN, tb, 0, st, Bn, 3, 4, 0, 0, 0);
        hipLaunchKernelGGL(k_pad_to_nat<double>, gN, tb, 0, st, Bn, y_nat, 0);
    }
}

void launch_nodal_out(const Dev* dd, const Dev* hd, int field, double* out, hipStream_t st) {
    Batch Bn = make_batch({dd}, {hd->Nnode}, TPB);
    if (field == 2) {
        if (hd->mixed) hipLaunchKernelGGL(k_pad_to_nat<float>, dim3(Bn.pfx[1]), dim3(TPB), 0, st, Bn, out, 2);
        else hipLaunchKernelGGL(k_pad_to_nat<double>, dim3(Bn.pfx[1]), dim3(TPB), 0, st, Bn, out, 2);
    } else {
        hipLaunchKernelGGL(k_nodal_scalar_out, dim3(Bn.pfx[1]), dim3(TPB), 0, st, Bn, out, field);
    }
}

void launch_residual_out(const Dev* dd, const Dev* hd, double* out, hipStream_t st) {
    Batch Bn = make_batch({dd}, {hd->Nnode}, TPB);
    hipLaunchKernelGGL(k_pad_to_nat<double>, dim3(Bn.pfx[1]), dim3(TPB), 0, st, Bn, out, 1);
}

void launch_set_state(const Dev* dd, const Dev* hd, const double* U, const double* P, hipStream_t st) {
    Batch Bn = make_batch({dd}, {hd->Nnode}, TPB);
    hipLaunchKernelGGL(k_set_state, dim3(Bn.pfx[1]), dim3(TPB), 0, st, Bn, U, P);
}

}  // namespace ppm
