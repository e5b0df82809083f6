// Linear solver of each Newton iteration (Sec. 3.4): BiCGStab on the fixed-stencil block rows
// of the Jacobian, right-preconditioned by the block upper-triangular operator
//       P = [ A  B1 ]      applied as   z_p = S^-1 r_p,   z_u = A^-1 (r_u - B1 z_p)
//           [ 0  S  ]
// (the Schur complement first, then A, as in the paper's solver).  The inverses are one
// geometric-multigrid V-cycle each on the structured background grid: damped block-Jacobi
// smoothing, bilinear transfer, Galerkin coarse operators R A P built on the device, a dense
// inverse on the coarsest level.  S is approximated by the fixed-stress form
// C + C_stab + (c_t / K) M_p (M_p lumped, K = lam + 2G/dim), or, as an option for problems whose
// displacement block is dominated by inertia, by C - B2 diag(A)^-1 B1 (k_schur_diag).
//
// Precision T is double (FP64 path) or float (mixed path: Jacobian, SpMV, preconditioner and
// Krylov vectors in FP32; dot products accumulate in FP64; the Newton update is FP64).
// Every BiCGStab scalar stays on the device; a per-problem flag stops finished problems.
#include "solver_common.hpp"
#include "launch.hpp"

namespace ppm {

// ---------------------------------------------------------------------------------------------
// SpMV on the fixed-stencil block rows: y = J x, optional dot products
//   mode 1: partial (a, y)        mode 2: partials (y, a), (y, y)
// FP64: one thread per scalar row (node, component a).  Wavefront W of the launch takes
// component a = W mod b of the 64 consecutive nodes 64 (W div b) + lane, so each of its S b
// Jacobian loads is one contiguous 64-row run, and b times as many wavefronts as with a thread
// per node keep enough bytes in flight (2D config: 78 -> 54 us).  FP32: one thread per node and
// all its b rows (half the bytes per load; splitting measured slower there).  Launched with
// spmv_blocks(dim, Nnode, T is double) blocks.
// ---------------------------------------------------------------------------------------------
template <int DIM, int R, typename T>
__global__ void __launch_bounds__(TPB) k_spmv(Batch B, int ix, int iy, int ia, int mode, int check_done) {
    PROB_PROLOGUE
    constexpr bool SPLIT = sizeof(T) == 8;
    constexpr int BS = DIM + 1;
    constexpr int NA = SPLIT ? 1 : BS;   // component rows per thread
    constexpr int SW = 2 * R + 1;
    constexpr int S = DIM == 2 ? SW * SW : SW * SW * SW;
    double dots[2] = {0.0, 0.0};
    int a0 = 0;
    int64_t row = tid;
    if (SPLIT) {
        const int64_t W = lb * (TPB / 64) + threadIdx.x / 64;
        a0 = (int)(W % BS);
        row = (W / BS) * 64 + (threadIdx.x & 63);
    }
    bool skip = check_done && krylov_done(d);
    if (!skip && row < d->Nnode) {
        void* const vecs[10] = {d->kx, d->kr, d->kh, d->kp, d->kv, d->ks, d->kt, d->kph, d->ksh, d->kbt};
        const T* __restrict__ x = vp<T>(vecs[ix]);
        T* __restrict__ y = vp<T>(vecs[iy]);
        const T* __restrict__ J = vp<T>(d->J);
        int c[3];
        real_coords(row, d->nn, DIM, c);
        const int64_t pn = padded(c, d->np1, R, DIM);
        double acc[NA];
#pragma unroll
        for (int i = 0; i < NA; ++i) acc[i] = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int64_t pk = pn + stencil_offset(s, R, DIM, d->np1);
            T xv[BS];
#pragma unroll
            for (int cc = 0; cc < BS; ++cc) xv[cc] = x[pk * BS + cc];
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const int a = a0 + i;
                T t = 0;
#pragma unroll
                for (int cc = 0; cc < BS; ++cc) {
                    const T* jp = &J[jidx<DIM>((s * BS + a) * BS + cc, row, S * BS * BS, d->Nnode)];
                    // 3D: the Jacobian (GBs) streams from HBM, keep it out of the caches; 2D: it
                    // mostly stays in the Infinity Cache between launches, plain loads measured faster
                    t += (DIM == 3 ? __builtin_nontemporal_load(jp) : *jp) * xv[cc];
                }
                acc[i] += (double)t;
            }
        }
#pragma unroll
        for (int i = 0; i < NA; ++i) y[pn * BS + a0 + i] = (T)acc[i];
        if (mode) {
            const T* __restrict__ av = vp<T>(vecs[ia]);
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const double yv = (double)(T)acc[i];
                dots[0] += (double)av[pn * BS + a0 + i] * yv;
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

// The vector kernels take the block size at compile time and read every operand of a node
// before writing, through restrict-qualified pointers, so the loads of all b components are in
// flight together.

// x = x_best = 0, r = rhat = -R, p = v = 0; partial (r, r)
template <int BS, typename T>
__global__ void __launch_bounds__(TPB) k_bicg_init(Batch B) {
    PROB_PROLOGUE
    double v[1] = {0.0};
    if (tid < d->Nnode) {
        const int64_t k0 = node_pad<T>(d, tid) * BS;
        const double* __restrict__ Rv = d->Rv;
        T* __restrict__ x = vp<T>(d->kx);
        T* __restrict__ r = vp<T>(d->kr);
        T* __restrict__ h = vp<T>(d->kh);
        T* __restrict__ pp = vp<T>(d->kp);
        T* __restrict__ vv = vp<T>(d->kv);
        T* __restrict__ xb = vp<T>(d->kxb);
        T rv[BS];
#pragma unroll
        for (int a = 0; a < BS; ++a) rv[a] = (T)(-Rv[k0 + a]);
#pragma unroll
        for (int a = 0; a < BS; ++a) {
            x[k0 + a] = 0;
            xb[k0 + a] = 0;
            r[k0 + a] = rv[a];
            h[k0 + a] = rv[a];
            pp[k0 + a] = 0;
            vv[k0 + a] = 0;
            v[0] += (double)rv[a] * (double)rv[a];
        }
    }
    block_partials<1>(d, lb, v);
}

// p = r + beta (p - omega v); on a restart rhat = p = r
template <int BS, typename T>
__global__ void __launch_bounds__(TPB) k_bicg_p(Batch B) {
    PROB_PROLOGUE
    if (krylov_done(d) || tid >= d->Nnode) return;
    const int64_t k0 = node_pad<T>(d, tid) * BS;
    T* __restrict__ p = vp<T>(d->kp);
    const T* __restrict__ r = vp<T>(d->kr);
    if (d->scal[SC_RESTART] == 2.0) {
        T* __restrict__ h = vp<T>(d->kh);
        T rv[BS];
#pragma unroll
        for (int a = 0; a < BS; ++a) rv[a] = r[k0 + a];
#pragma unroll
        for (int a = 0; a < BS; ++a) {
            p[k0 + a] = rv[a];
            h[k0 + a] = rv[a];
        }
        return;
    }
    const T beta = (T)d->scal[SC_BETA], om = (T)d->scal[SC_OMEGA];
    const T* __restrict__ v = vp<T>(d->kv);
    T pv[BS], rv[BS], vv[BS];
#pragma unroll
    for (int a = 0; a < BS; ++a) {
        pv[a] = p[k0 + a];
        rv[a] = r[k0 + a];
        vv[a] = v[k0 + a];
    }
#pragma unroll
    for (int a = 0; a < BS; ++a) p[k0 + a] = rv[a] + beta * (pv[a] - om * vv[a]);
}

// BiCGStab breakdown ((rhat, v) = 0, rho = 0 or omega = 0 with the residual still finite and
// above the tolerance): restart from the current iterate with rhat = p = r, at most
// MAX_RESTARTS times per solve; after that the solve ends (breakdown reported).
constexpr int MAX_RESTARTS = 8;

__device__ __forceinline__ bool can_restart(const double* sc) {
    const double rr = sc[SC_RR];
    return isfinite(rr) && rr > 0.0 && sc[SC_NRESTART] < (double)MAX_RESTARTS;
}

// alpha = rho / (rhat, v) from the SpMV's partials (each block reduces them itself, in the
// order of the scalar kernel, so all blocks agree; block 0 records alpha), then s = r - alpha v.
// A zero or non-finite (rhat, v) is a breakdown: the rest of the iteration is skipped (done
// flag) and the scalar kernel sets up a restart, or ends the solve.
template <int BS, typename T>
__global__ void __launch_bounds__(TPB) k_bicg_s(Batch B) {
    PROB_PROLOGUE
    if (krylov_done(d)) return;
    double s0, s1;
    sum_partials(d, spmv_blocks(d->dim, d->Nnode, !d->mixed), &s0, &s1);
    (void)s1;
    const bool brk = s0 == 0.0 || !isfinite(s0);
    const double alpha = brk ? 0.0 : d->scal[SC_RHO] / s0;
    if (lb == 0 && threadIdx.x == 0) {
        d->scal[SC_RV] = s0;
        if (brk) {
            if (can_restart(d->scal)) d->scal[SC_RESTART] = 1.0;
            else d->scal[SC_BREAK] = 1.0;
            d->scal[SC_DONE] = 1.0;
        } else {
            d->scal[SC_ALPHA] = alpha;
        }
    }
    if (brk || tid >= d->Nnode) return;
    const int64_t k0 = node_pad<T>(d, tid) * BS;
    const T al = (T)alpha;
    const T* __restrict__ r = vp<T>(d->kr);
    const T* __restrict__ vv = vp<T>(d->kv);
    T* __restrict__ sp = vp<T>(d->ks);
    T rv[BS], w[BS];
#pragma unroll
    for (int a = 0; a < BS; ++a) {
        rv[a] = r[k0 + a];
        w[a] = vv[k0 + a];
    }
#pragma unroll
    for (int a = 0; a < BS; ++a) sp[k0 + a] = rv[a] - al * w[a];
}

// omega = (t, s) / (t, t) from the SpMV's partials (reduced by every block, as in k_bicg_s;
// t = 0 means s is already the exact residual of x + alpha ph: omega = 0), then
// x += alpha ph + omega sh; r = s - omega t; partials (rhat, r), (r, r) in slots 2 and 3 (slots
// 0 and 1 hold the SpMV's, which other blocks may still be reading).
template <int BS, typename T>
__global__ void __launch_bounds__(TPB) k_bicg_xr(Batch B) {
    PROB_PROLOGUE
    if (krylov_done(d)) return;
    double ts, tt;
    sum_partials(d, spmv_blocks(d->dim, d->Nnode, !d->mixed), &ts, &tt);
    const double omega = (tt == 0.0 || !isfinite(tt)) ? 0.0 : ts / tt;
    if (lb == 0 && threadIdx.x == 0) {
        d->scal[SC_TS] = ts;
        d->scal[SC_TT] = tt;
        d->scal[SC_OMEGA] = omega;
    }
    double v[2] = {0.0, 0.0};
    if (tid < d->Nnode) {
        const int64_t k0 = node_pad<T>(d, tid) * BS;
        const T al = (T)d->scal[SC_ALPHA], om = (T)omega;
        T* __restrict__ x = vp<T>(d->kx);
        T* __restrict__ r = vp<T>(d->kr);
        const T* __restrict__ ph = vp<T>(d->kph);
        const T* __restrict__ sh = vp<T>(d->ksh);
        const T* __restrict__ sp = vp<T>(d->ks);
        const T* __restrict__ tp = vp<T>(d->kt);
        const T* __restrict__ h = vp<T>(d->kh);
        T xv[BS], pv[BS], qv[BS], sv[BS], tv[BS], hv[BS];
#pragma unroll
        for (int a = 0; a < BS; ++a) {
            xv[a] = x[k0 + a];
            pv[a] = ph[k0 + a];
            qv[a] = sh[k0 + a];
            sv[a] = sp[k0 + a];
            tv[a] = tp[k0 + a];
            hv[a] = h[k0 + a];
        }
#pragma unroll
        for (int a = 0; a < BS; ++a) {
            x[k0 + a] = xv[a] + (al * pv[a] + om * qv[a]);
            const T rr = sv[a] - om * tv[a];
            r[k0 + a] = rr;
            v[0] += (double)hv[a] * (double)rr;
            v[1] += (double)rr * (double)rr;
        }
    }
    block_partials<2>(d, lb, v, 2);
}

// scalar updates, one block per problem; stage:
//   0 after init: rho = (r,r), tol2, alpha = omega = 1, beta = 0   (partials in slot 0)
//   3 after x, r: beta, rho, convergence                           (partials in slots 2, 3)
// (alpha and omega are formed by k_bicg_s and k_bicg_xr from the SpMV partials)
__global__ void k_bicg_scalars(Batch B, int stage, double rtol, int maxit) {
    const int q = blockIdx.x;
    const Dev* d = B.d[q];
    // every thread reads the flags before thread 0 may change them, so that the block decides
    // uniformly
    const bool done0 = krylov_done(d);
    const double rst0 = d->scal[SC_RESTART];
    __syncthreads();
    if (stage != 0 && done0 && rst0 != 1.0) return;
    if (stage != 0 && rst0 == 1.0) {
        // breakdown in k_bicg_s: x and r are those of the previous iteration (RR their norm)
        if (threadIdx.x == 0) {
            double* sc = d->scal;
            sc[SC_ITER] += 1.0;
            sc[SC_NRESTART] += 1.0;
            sc[SC_RHO] = sc[SC_RR];
            sc[SC_RESTART] = 2.0;
            sc[SC_DONE] = sc[SC_ITER] >= (double)maxit ? 1.0 : 0.0;
        }
        return;
    }
    __shared__ double sh[2][TPB];
    const int64_t nblk = (d->Nnode + TPB - 1) / TPB;
    const int slot = stage == 3 ? 2 : 0;
    double a = 0.0, b2 = 0.0;
    for (int64_t i = threadIdx.x; i < nblk; i += TPB) {
        a += d->partial[i * 4 + slot];
        b2 += d->partial[i * 4 + slot + 1];
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
        sc[SC_BEST] = s0;
        sc[SC_SREF] = s0;
        sc[SC_SITER] = 0.0;
        sc[SC_RESTART] = 0.0;
        sc[SC_NRESTART] = 0.0;
        sc[SC_DONE] = (s0 == 0.0 || maxit <= 0) ? 1.0 : 0.0;
    } else {
        double rho_new = s0;
        sc[SC_RR] = s1;
        sc[SC_ITER] += 1.0;
        sc[SC_RESTART] = 0.0;   // a restart set up by the previous iteration has been applied
        bool conv = s1 <= sc[SC_TOL2];
        bool brk = (rho_new == 0.0 || sc[SC_OMEGA] == 0.0 || !isfinite(s1));
        if (!conv && brk && sc[SC_ITER] < (double)maxit && can_restart(sc)) {
            sc[SC_NRESTART] += 1.0;
            sc[SC_RHO] = s1;   // (rhat, r) with rhat = r
            sc[SC_RESTART] = 2.0;
            return;
        }
        if (!conv && brk) sc[SC_BREAK] = 1.0;
        if (conv || brk || sc[SC_ITER] >= (double)maxit) {
            sc[SC_DONE] = 1.0;
            return;
        }
        sc[SC_BETA] = (rho_new / sc[SC_RHO]) * (sc[SC_ALPHA] / sc[SC_OMEGA]);
        sc[SC_RHO] = rho_new;
    }
}

// Best iterate and stagnation.  BiCGStab's residual is not monotone, and in FP32 it can stall
// above the tolerance or grow without bound once rounding has taken over the recurrences (the
// near-incompressible blocks of the mixed path).  At the end of every chunk of iterations the
// iterate is copied to x_best when its residual is the smallest seen so far at a chunk end
// (k_bicg_keep, then k_bicg_keep_scal records it); a solve that ends above its tolerance hands
// the better of x and x_best to the Newton update (k_bicg_pick).  The mixed path also stops a
// solve whose residual norm has not halved in STALL_ITERS iterations: the Newton update then
// takes x_best under the residual-decrease test of the outer loop, and the next Newton iteration
// refines it.
constexpr int STALL_ITERS = 256;

__device__ __forceinline__ bool keep_best(const Dev* d) {
    const double rr = d->scal[SC_RR];
    return isfinite(rr) && rr < d->scal[SC_BEST];
}

template <int BS, typename T>
__global__ void __launch_bounds__(TPB) k_bicg_keep(Batch B) {
    PROB_PROLOGUE
    if (krylov_done(d) || !keep_best(d) || tid >= d->Nnode) return;
    const int64_t k0 = node_pad<T>(d, tid) * BS;
    const T* __restrict__ x = vp<T>(d->kx);
    T* __restrict__ xb = vp<T>(d->kxb);
    T xv[BS];
#pragma unroll
    for (int a = 0; a < BS; ++a) xv[a] = x[k0 + a];
#pragma unroll
    for (int a = 0; a < BS; ++a) xb[k0 + a] = xv[a];
}

// one block per problem, after k_bicg_keep (which reads SC_BEST)
__global__ void k_bicg_keep_scal(Batch B) {
    const Dev* d = B.d[blockIdx.x];
    if (threadIdx.x != 0 || krylov_done(d)) return;
    double* sc = d->scal;
    const double rr = sc[SC_RR];
    if (keep_best(d)) sc[SC_BEST] = rr;
    if (rr < 0.25 * sc[SC_SREF]) {
        sc[SC_SREF] = rr;
        sc[SC_SITER] = sc[SC_ITER];
    } else if (d->mixed && sc[SC_ITER] - sc[SC_SITER] >= (double)STALL_ITERS) {
        sc[SC_DONE] = 1.0;
    }
}

// after the solve: a problem that ended above its tolerance takes x_best when x is worse
template <int BS, typename T>
__global__ void __launch_bounds__(TPB) k_bicg_pick(Batch B) {
    PROB_PROLOGUE
    const double rr = d->scal[SC_RR];
    if (rr <= d->scal[SC_TOL2] || rr <= d->scal[SC_BEST] || tid >= d->Nnode) return;
    const int64_t k0 = node_pad<T>(d, tid) * BS;
    T* __restrict__ x = vp<T>(d->kx);
    const T* __restrict__ xb = vp<T>(d->kxb);
    T xv[BS];
#pragma unroll
    for (int a = 0; a < BS; ++a) xv[a] = xb[k0 + a];
#pragma unroll
    for (int a = 0; a < BS; ++a) x[k0 + a] = xv[a];
}

// X += s x (Newton update, FP64; s = 1, or a negative fraction that takes back part of the last
// update)
template <typename T>
__global__ void __launch_bounds__(TPB) k_newton_update(Batch B, double s) {
    PROB_PROLOGUE
    if (tid >= d->Nnode) return;
    const int64_t pn = node_pad<T>(d, tid);
    const int bs = d->b;
    for (int a = 0; a < bs; ++a) {
        int64_t k = pn * bs + a;
        if (d->dfree[k]) d->X[k] += s * (double)vp<T>(d->kx)[k];
    }
}

static std::vector<int64_t> spmv_grid(const Group& g) {
    std::vector<int64_t> v;
    for (size_t q = 0; q < g.nnode.size(); ++q) v.push_back(spmv_blocks(g.dim, g.nnode[q], !g.mixed));
    return v;
}

template <int DIM, int R, typename T>
static void krylov_iters_t(const Group& g, const std::vector<const Dev*>& hc, int iters, double rtol, int maxit,
                           hipStream_t st) {
    Batch Bn = make_batch(g.ddev, g.nnode, TPB);
    Batch Bs = make_batch_blocks(g.ddev, spmv_grid(g));
    Batch B1 = make_batch_one_block(g.ddev);
    const dim3 gN(Bn.pfx[Bn.n]), gS(Bs.pfx[Bs.n]), tb(TPB);
    // vector ids: 0 x, 1 r, 2 rhat, 3 p, 4 v, 5 s, 6 t, 7 ph, 8 sh
    for (int it = 0; it < iters; ++it) {
        hipLaunchKernelGGL((k_bicg_p<DIM + 1, T>), gN, tb, 0, st, Bn);
        launch_precond_apply(g, hc, 3, 7, st);
        PPM_TIMED(KT_SPMV, st, hipLaunchKernelGGL((k_spmv<DIM, R, T>), gS, tb, 0, st, Bs, 7, 4, 2, 1, 1));
        hipLaunchKernelGGL((k_bicg_s<DIM + 1, T>), gN, tb, 0, st, Bn);
        launch_precond_apply(g, hc, 5, 8, st);
        PPM_TIMED(KT_SPMV, st, hipLaunchKernelGGL((k_spmv<DIM, R, T>), gS, tb, 0, st, Bs, 8, 6, 5, 2, 1));
        hipLaunchKernelGGL((k_bicg_xr<DIM + 1, T>), gN, tb, 0, st, Bn);
        hipLaunchKernelGGL(k_bicg_scalars, dim3(B1.n), tb, 0, st, B1, 3, rtol, maxit);
    }
    hipLaunchKernelGGL((k_bicg_keep<DIM + 1, T>), gN, tb, 0, st, Bn);
    hipLaunchKernelGGL(k_bicg_keep_scal, dim3(B1.n), dim3(64), 0, st, B1);
}

void launch_krylov_init(const Group& g, double rtol, int maxit, hipStream_t st) {
    Batch Bn = make_batch(g.ddev, g.nnode, TPB);
    Batch B1 = make_batch_one_block(g.ddev);
    const dim3 gN(Bn.pfx[Bn.n]), tb(TPB);
    if (g.dim == 2) {
        if (g.mixed) hipLaunchKernelGGL((k_bicg_init<3, float>), gN, tb, 0, st, Bn);
        else hipLaunchKernelGGL((k_bicg_init<3, double>), gN, tb, 0, st, Bn);
    } else {
        if (g.mixed) hipLaunchKernelGGL((k_bicg_init<4, float>), gN, tb, 0, st, Bn);
        else hipLaunchKernelGGL((k_bicg_init<4, double>), gN, tb, 0, st, Bn);
    }
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

void launch_krylov_pick(const Group& g, hipStream_t st) {
    Batch Bn = make_batch(g.ddev, g.nnode, TPB);
    const dim3 gN(Bn.pfx[Bn.n]), tb(TPB);
    if (g.dim == 2) {
        if (g.mixed) hipLaunchKernelGGL((k_bicg_pick<3, float>), gN, tb, 0, st, Bn);
        else hipLaunchKernelGGL((k_bicg_pick<3, double>), gN, tb, 0, st, Bn);
    } else {
        if (g.mixed) hipLaunchKernelGGL((k_bicg_pick<4, float>), gN, tb, 0, st, Bn);
        else hipLaunchKernelGGL((k_bicg_pick<4, double>), gN, tb, 0, st, Bn);
    }
}

void launch_newton_update(const Group& g, hipStream_t st, double s) {
    Batch Bn = make_batch(g.ddev, g.nnode, TPB);
    if (g.mixed) hipLaunchKernelGGL(k_newton_update<float>, dim3(Bn.pfx[Bn.n]), dim3(TPB), 0, st, Bn, s);
    else hipLaunchKernelGGL(k_newton_update<double>, dim3(Bn.pfx[Bn.n]), dim3(TPB), 0, st, Bn, s);
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
        else if (which == 3) v = d->X[k];
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
    Batch Bs = make_batch_blocks({dd}, {spmv_blocks(hd->dim, hd->Nnode, !hd->mixed)});
    const dim3 gN(Bn.pfx[1]), gS(Bs.pfx[1]), tb(TPB);
    int R = hd->R;
    if (hd->mixed) {
        hipLaunchKernelGGL(k_nat_to_pad<float>, gN, tb, 0, st, Bn, v_nat, 0);
        if (hd->dim == 2 && R == 1) hipLaunchKernelGGL((k_spmv<2, 1, float>), gS, tb, 0, st, Bs, 3, 4, 0, 0, 0);
        else if (hd->dim == 2) hipLaunchKernelGGL((k_spmv<2, 2, float>), gS, tb, 0, st, Bs, 3, 4, 0, 0, 0);
        else hipLaunchKernelGGL((k_spmv<3, 1, float>), gS, tb, 0, st, Bs, 3, 4, 0, 0, 0);
        hipLaunchKernelGGL(k_pad_to_nat<float>, gN, tb, 0, st, Bn, y_nat, 0);
    } else {
        hipLaunchKernelGGL(k_nat_to_pad<double>, gN, tb, 0, st, Bn, v_nat, 0);
        if (hd->dim == 2 && R == 1) hipLaunchKernelGGL((k_spmv<2, 1, double>), gS, tb, 0, st, Bs, 3, 4, 0, 0, 0);
        else if (hd->dim == 2) hipLaunchKernelGGL((k_spmv<2, 2, double>), gS, tb, 0, st, Bs, 3, 4, 0, 0, 0);
        else hipLaunchKernelGGL((k_spmv<3, 1, double>), gS, tb, 0, st, Bs, 3, 4, 0, 0, 0);
        hipLaunchKernelGGL(k_pad_to_nat<double>, gN, tb, 0, st, Bn, y_nat, 0);
    }
}

void launch_nodal_out(const Dev* dd, const Dev* hd, int field, double* out, hipStream_t st) {
    Batch Bn = make_batch({dd}, {hd->Nnode}, TPB);
    if (field == 3) {
        hipLaunchKernelGGL(k_pad_to_nat<double>, dim3(Bn.pfx[1]), dim3(TPB), 0, st, Bn, out, 3);
    } else if (field == 2) {
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
