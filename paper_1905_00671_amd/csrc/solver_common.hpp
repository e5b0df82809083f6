// Device helpers shared by the Krylov and multigrid kernels: padded-grid indexing, stencil
// offsets, deterministic block reductions, operator access and per-problem vector references.
#pragma once
#include "ppmpm_internal.hpp"

namespace ppm {

#define PROB_PROLOGUE                                   \
    const int q = batch_find(B, blockIdx.x);            \
    const Dev* __restrict__ d = B.d[q];                 \
    const int64_t lb = blockIdx.x - B.pfx[q];           \
    const int64_t tid = lb * blockDim.x + threadIdx.x;

template <typename T>
__device__ __forceinline__ T* vp(void* p) { return (T*)p; }

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

// block reduction of NV values into partial[lb*4 + slot + k] (fixed tree order: deterministic)
template <int NV>
__device__ __forceinline__ void block_partials(const Dev* d, int64_t lb, const double* v, int slot = 0) {
    __shared__ double sh[NV][TPB];
    for (int k = 0; k < NV; ++k) sh[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int off = TPB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int k = 0; k < NV; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < NV; ++k) d->partial[lb * 4 + slot + k] = sh[k][0];
}

// Sum over nblk blocks of partial[i*4 + k], k < 2, returned to every thread of the block: thread t
// adds blocks t, t + TPB, ..., then a fixed tree, so every block (and the one-block scalar kernel)
// gets the same bits.  Ends with a barrier; the block's threads must all call it.
__device__ __forceinline__ void sum_partials(const Dev* d, int64_t nblk, double* s0, double* s1) {
    __shared__ double sh[2][TPB];
    double a = 0.0, b = 0.0;
    for (int64_t i = threadIdx.x; i < nblk; i += TPB) {
        a += d->partial[i * 4 + 0];
        b += d->partial[i * 4 + 1];
    }
    sh[0][threadIdx.x] = a;
    sh[1][threadIdx.x] = b;
    __syncthreads();
    for (int off = TPB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + off];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    *s0 = sh[0][0];
    *s1 = sh[1][0];
    __syncthreads();
}

__device__ __forceinline__ bool krylov_done(const Dev* d) { return d->scal[SC_DONE] != 0.0; }

// Operator entry (row, stencil s, a, c) of family fam (0: A, block dim; 1: S, block 1) on level l.
// Level 0 reads the Jacobian's stored blocks (row-blocked layout, see jidx); coarser levels their
// Galerkin operators [S][B][B][nrow].  One index formula covers both:
//   (row >> sh) * bstride + e * estride + (row & mask).
template <typename T>
struct Op {
    const T* base;
    int64_t nrow;
    int BJ;   // block size of the storage
    int a0;   // first storage row/col of the family
    int sh;
    int64_t mask, estride, bstride;
    __device__ __forceinline__ double at(int s, int a, int c, int64_t row) const {
        const int64_t e = (int64_t)(s * BJ + a + a0) * BJ + c + a0;
        return (double)base[(row >> sh) * bstride + e * estride + (row & mask)];
    }
};

template <typename T>
__device__ __forceinline__ Op<T> op_of(const Dev* d, int fam, int l) {
    Op<T> o;
    if (l == 0 && !(fam == 1 && d->schur)) {
        o.base = (const T*)d->J;
        o.nrow = d->Nnode;
        o.BJ = d->b;
        o.a0 = fam == 0 ? 0 : d->dim;
        const bool blk = d->dim == 3;   // layout of jidx
        o.sh = blk ? 6 : 62;
        o.mask = blk ? (int64_t)(JB - 1) : ~(int64_t)0;
        o.estride = blk ? (int64_t)JB : d->Nnode;
        o.bstride = blk ? (int64_t)d->S * d->b * d->b * JB : 0;
    } else {
        o.base = (const T*)(fam == 0 ? d->lev[l].A : d->lev[l].Sm);
        o.nrow = d->lev[l].nrow;
        o.BJ = fam == 0 ? d->dim : 1;
        o.a0 = 0;
        o.sh = 62;
        o.mask = ~(int64_t)0;
        o.estride = o.nrow;
        o.bstride = 0;
    }
    return o;
}

// fixed-stress diagonal of the Schur approximation on level 0 (zero on non-free pressure dofs):
// c_t / K M_p.  Newmark problems add the inertia of the displacement block to the modulus,
// K = K_fs + kin rho_i h^2 / (beta dt^2) with the nodal density rho_i = M_i / M_p,i: a pressure
// mode of wavenumber xi sees A^-1 ~ 1 / (K_fs xi^2 + rho / (beta dt^2)); kin is set by Krylov
// counts (1: the grid's shortest modes see a few times less inertia than this)
__device__ __forceinline__ double fs_term(const Dev* d, int64_t pn) {
    // the diagonal-inverse form stores its level-0 operator whole (k_schur_diag)
    if (d->schur || !d->dfree[pn * d->b + d->dim]) return 0.0;
    double K = d->Kfs;
    if (d->dyn) K += d->kin * d->M[pn] / d->Mp[pn] * d->h * d->h / (d->beta * d->dt * d->dt);
    return d->ct / K * d->Mp[pn];
}

__device__ __forceinline__ double mask0(const Dev* d, int fam, int64_t pn, int comp) {
    return d->dfree[pn * d->b + (fam == 0 ? comp : d->dim)] ? 1.0 : 0.0;
}

// Symbolic vector reference resolved per problem inside the kernels, so that one launch serves
// every problem of a batch: kinds 0..8 are the Krylov vectors (x r rhat p v s t ph sh, block b,
// component offset `off`), 9 is the rhs of the A cycle on level 0 (block dim), 10/11/12 are the
// level iterate / residual / right-hand side of the family being cycled (block BB), 13 is where
// the up-sweep leaves the level's correction: the iterate buffer on the coarsest level (written
// by the dense solve), the residual buffer on the others (the fused post-smoother writes there).
struct VRef {
    int kind;
    int off;
};
enum { VK_BT = 9, VK_LX = 10, VK_LR = 11, VK_LB = 12, VK_SOL = 13 };

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
        int kind = v.kind;
        if (kind == VK_SOL) kind = l == d->nlev - 1 ? VK_LX : VK_LR;
        void* p;
        if (kind == VK_LX) p = fam == 0 ? L.xa : L.xs;
        else if (kind == VK_LR) p = fam == 0 ? L.ra : L.rs;
        else p = fam == 0 ? L.ba : L.bsv;
        o.p = (T*)p;
        o.stride = BB;
    }
    return o;
}

}  // namespace ppm
