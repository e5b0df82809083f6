// Consistent-mass P2G (eq. map-from-particles-to-nodes-consistent) and tractions carried by
// material points (the Neumann load of the strip footing, Sec. 5.2).
//
// Consistent mapping: the nodal fields f solve sum_j M_ij f_j = b_i = sum_mp S_i m f_mp with the
// consistent mass matrix M_ij = sum_mp S_i S_j m.  Nodes whose lumped mass M_i is below
// LIGHT_NODE times the largest nodal mass of the problem ("light" nodes, barely reached by a
// point domain) keep the lumped value b_i / M_i and enter the other ("heavy") rows as known
// values: M_HH f_H = b_H - M_HL f_L.  The rows of M are gathered per node over the fixed stencil
// (no atomics, as the lumped P2G), and the system is solved by conjugate gradients with the
// lumped mass as preconditioner, every mapped field (p; v, a, pdot, pddot on dynamic steps) a
// column with its own scalars, starting from the lumped values.  Reductions are per-block
// partials in a fixed tree order, summed by a one-block kernel: the result does not depend on
// scheduling.
//
// Point tractions: point q carries the force F_q (traction times its share of the loaded
// boundary) on the face of its domain whose outward normal is the coordinate axis n_q; along that
// axis the grid's hat is evaluated on the face x_a + lp_a n_a, along the others the point's own
// 1D basis.  Each node gathers the forces of the loaded points in the buckets that can reach it,
// in the sort's order, so its sum is formed in the same order on every run.
#include "ppmpm_internal.hpp"
#include "launch.hpp"
#include "solver_common.hpp"

namespace ppm {

namespace {

constexpr double LIGHT_NODE = 1e-2;   // light-node threshold, relative to the largest nodal mass
constexpr double MASS_RTOL = 1e-13;   // ||r|| <= MASS_RTOL ||b_H|| per column
constexpr int MASS_MAXIT = 2000;
constexpr int MASS_CHECK = 8;         // iterations between host checks of the convergence flag

// per-column scalar slots in Dev::mscal (column c at c * MS_STRIDE)
enum : int { MS_RZ = 0, MS_ALPHA, MS_BETA, MS_TOL2, MS_DONE, MS_RR, MS_STRIDE = 8 };
// problem-wide slots after the MCOL column blocks
enum : int { MG_MAX = 0, MG_ALLDONE, MG_ITERS };

__device__ __forceinline__ double* mcol(const Dev* d, int c) { return d->mscal + c * MS_STRIDE; }
__device__ __forceinline__ double* mglob(const Dev* d) { return d->mscal + MCOL * MS_STRIDE; }

__device__ __forceinline__ void node_coords(const Dev* d, int64_t row, int* n) {
    n[0] = (int)(row % d->nn[0]);
    n[1] = (int)((row / d->nn[0]) % d->nn[1]);
    n[2] = d->dim == 3 ? (int)(row / ((int64_t)d->nn[0] * d->nn[1])) : 0;
}

// natural index of the stencil neighbour s of node n, or -1 outside the grid
template <int DIM, int R>
__device__ __forceinline__ int64_t stencil_nbr(const Dev* d, const int* n, int s) {
    constexpr int SW = 2 * R + 1;
    const int o[3] = {s % SW - R, (s / SW) % SW - R, DIM == 3 ? s / (SW * SW) - R : 0};
    int k[3];
    for (int a = 0; a < 3; ++a) {
        k[a] = n[a] + o[a];
        if (a < DIM && (k[a] < 0 || k[a] >= d->nn[a])) return -1;
    }
    return k[0] + (int64_t)d->nn[0] * (k[1] + (int64_t)d->nn[1] * k[2]);
}

// Sum of NV values over the block, fixed order (wavefront tree, then the waves in order); the
// result is valid in thread 0.  Every thread of the block must call it.
template <int NV>
__device__ __forceinline__ void block_sum(double* v, double* out) {
    __shared__ double sh[NV][TPB / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) sh[k][wave] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int w = 0; w < TPB / 64; ++w) s += sh[k][w];
            out[k] = s;
        }
    __syncthreads();
}

// Sum over the problem's node blocks of partial slots off .. off + nv_used - 1 (NV slots per
// block), in thread 0: thread t adds blocks t, t + TPB, ..., then block_sum.
template <int NV>
__device__ __forceinline__ void sum_blocks(const Dev* d, int64_t nblk, int nv_used, double* out, int off = 0) {
    double v[NV];
    for (int k = 0; k < NV; ++k) v[k] = 0.0;
    for (int64_t i = threadIdx.x; i < nblk; i += TPB)
        for (int k = 0; k < nv_used; ++k) v[k] += d->mpart[i * NV + off + k];
    block_sum<NV>(v, out);
}

__device__ __forceinline__ int64_t node_blocks(const Dev* d) { return (d->Nnode + TPB - 1) / TPB; }

// NS consecutive partial slots first .. first + NS - 1 summed over the problem's node blocks, in
// thread 0: per slot the same additions in the same order as sum_blocks<3 MCOL>
template <int NS>
__device__ __forceinline__ void sum_slots(const Dev* d, int64_t nblk, int first, double* out) {
    double v[NS];
    for (int k = 0; k < NS; ++k) v[k] = 0.0;
    for (int64_t i = threadIdx.x; i < nblk; i += TPB)
        for (int k = 0; k < NS; ++k) v[k] += d->mpart[i * 3 * MCOL + first + k];
    block_sum<NS>(v, out);
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// consistent mass rows: per node, gather over the buckets whose points reach it
// ---------------------------------------------------------------------------------------------
template <int DIM, int SHAPE>
__global__ void __launch_bounds__(TPB) k_mass_rows(Batch B) {
    PROB_PROLOGUE
    if (tid >= d->Nnode || !d->cons) return;
    constexpr int WB = SHAPE ? 3 : 2;
    constexpr int R = SHAPE ? 2 : 1;
    constexpr int SW = 2 * R + 1;
    constexpr int S = DIM == 2 ? SW * SW : SW * SW * SW;
    int n[3];
    node_coords(d, tid, n);
    const double* P = d->pw;
    const int64_t s = d->ps;
    int clo[3] = {0, 0, 0}, chi[3] = {0, 0, 0};
    for (int a = 0; a < DIM; ++a) {
        clo[a] = n[a] - (SHAPE ? 2 : 1);
        chi[a] = n[a] + (SHAPE ? 1 : 0);
        clo[a] = clo[a] < 0 ? 0 : clo[a];
        chi[a] = chi[a] > d->nc[a] - 1 ? d->nc[a] - 1 : chi[a];
    }
    double row[S];
    for (int e = 0; e < S; ++e) row[e] = 0.0;
    for (int cz = (DIM == 3 ? clo[2] : 0); cz <= (DIM == 3 ? chi[2] : 0); ++cz)
        for (int cy = clo[1]; cy <= chi[1]; ++cy)
            for (int cx = clo[0]; cx <= chi[0]; ++cx) {
                const int64_t c = cx + (int64_t)d->nc[0] * (cy + (int64_t)d->nc[1] * cz);
                const int p0 = d->cstart[c], p1 = d->cstart[c + 1];
                for (int i = p0; i < p1; ++i) {
                    double w[DIM][3], dw[3], s0v[3];
                    int li[3] = {0, 0, 0};
                    bool in = true;
                    for (int a = 0; a < DIM; ++a) {
                        const int base = basis_1d<SHAPE>(P[(PX + a) * s + i], P[(PLP + a) * s + i], d->x0[a], d->h,
                                                          d->nc[a], w[a], dw, s0v);
                        li[a] = n[a] - base;
                        if (li[a] < 0 || li[a] >= WB) in = false;
                    }
                    if (!in) continue;
                    double Si = P[PM * s + i];
                    for (int a = 0; a < DIM; ++a) Si *= w[a][li[a]];
                    if (Si == 0.0) continue;
                    // columns: the other nodes of the point's window, at stencil offsets lk - li
                    for (int e = 0; e < S; ++e) {
                        const int o[3] = {e % SW - R, (e / SW) % SW - R, DIM == 3 ? e / (SW * SW) - R : 0};
                        double Sk = 1.0;
                        for (int a = 0; a < DIM; ++a) {
                            const int lk = li[a] + o[a];
                            Sk = (lk >= 0 && lk < WB) ? Sk * w[a][lk] : 0.0;
                        }
                        row[e] += Si * Sk;
                    }
                }
            }
    for (int e = 0; e < S; ++e) d->mrow[e * d->Nnode + tid] = row[e];
}

__global__ void k_mass_clear(Batch B) {
    const Dev* d = B.d[blockIdx.x];
    if (!d->cons) return;
    for (int k = threadIdx.x; k < MCOL * MS_STRIDE + 8; k += blockDim.x) d->mscal[k] = 0.0;
}

// largest nodal mass (non-negative doubles order like their bit patterns)
__global__ void __launch_bounds__(TPB) k_mass_max(Batch B) {
    PROB_PROLOGUE
    if (!d->cons) return;   // uniform over the block (one problem per block)
    double m = 0.0;
    if (tid < d->Nnode) {
        int n[3];
        node_coords(d, tid, n);
        m = d->M[pad_index(d, n[0], n[1], n[2])];
    }
    block_max_nonneg(mglob(d) + MG_MAX, m);
}

// heavy / light split and the lumped start x = b / M
__global__ void __launch_bounds__(TPB) k_mass_init(Batch B) {
    PROB_PROLOGUE
    if (tid >= d->Nnode || !d->cons) return;
    int n[3];
    node_coords(d, tid, n);
    const double m = d->M[pad_index(d, n[0], n[1], n[2])];
    const bool act = m > 0.0;
    d->mheavy[tid] = (act && m >= LIGHT_NODE * mglob(d)[MG_MAX]) ? 1 : 0;
    for (int c = 0; c < d->ncol; ++c) d->mx[c * d->Nnode + tid] = act ? d->mb[c * d->Nnode + tid] / m : 0.0;
}

// r = b - M x, z = r / M_lumped, d = z on heavy rows (0 elsewhere); partials (r.z, r.r, b.b)
template <int DIM, int R>
__global__ void __launch_bounds__(TPB) k_mass_r0(Batch B) {
    PROB_PROLOGUE
    constexpr int SW = 2 * R + 1;
    constexpr int S = DIM == 2 ? SW * SW : SW * SW * SW;
    const int64_t N = d->Nnode;
    double v[3 * MCOL];
    for (int k = 0; k < 3 * MCOL; ++k) v[k] = 0.0;
    if (tid < N && d->cons && d->mheavy[tid]) {
        int n[3];
        node_coords(d, tid, n);
        const double m = d->M[pad_index(d, n[0], n[1], n[2])];
        for (int c = 0; c < d->ncol; ++c) {
            const double b = d->mb[c * N + tid];
            double r = b;
            for (int e = 0; e < S; ++e) {
                const int64_t k = stencil_nbr<DIM, R>(d, n, e);
                if (k >= 0) r -= d->mrow[e * N + tid] * d->mx[c * N + k];
            }
            const double z = r / m;
            d->mr[c * N + tid] = r;
            d->mz[c * N + tid] = z;
            d->md[c * N + tid] = z;
            v[3 * c] = r * z;
            v[3 * c + 1] = r * r;
            v[3 * c + 2] = b * b;
        }
    } else if (tid < N && d->cons) {
        for (int c = 0; c < d->ncol; ++c) d->mr[c * N + tid] = d->mz[c * N + tid] = d->md[c * N + tid] = 0.0;
    }
    double out[3 * MCOL];
    block_sum<3 * MCOL>(v, out);
    if (threadIdx.x == 0 && d->cons)
        for (int k = 0; k < 3 * MCOL; ++k) d->mpart[lb * 3 * MCOL + k] = out[k];
}

__global__ void k_mass_scal0(Batch B) {
    const Dev* d = B.d[blockIdx.x];
    if (!d->cons) return;
    double s[3 * MCOL];
    sum_blocks<3 * MCOL>(d, node_blocks(d), 3 * d->ncol, s);
    if (threadIdx.x == 0) {
        bool all = true;
        for (int c = 0; c < d->ncol; ++c) {
            double* m = mcol(d, c);
            m[MS_RZ] = s[3 * c];
            m[MS_RR] = s[3 * c + 1];
            m[MS_TOL2] = MASS_RTOL * MASS_RTOL * s[3 * c + 2];
            m[MS_DONE] = (s[3 * c + 2] == 0.0 || s[3 * c + 1] <= m[MS_TOL2]) ? 1.0 : 0.0;
            m[MS_ALPHA] = m[MS_BETA] = 0.0;
            all = all && m[MS_DONE] != 0.0;
        }
        mglob(d)[MG_ALLDONE] = all ? 1.0 : 0.0;
        mglob(d)[MG_ITERS] = 0.0;
    }
}

// One CG iteration is k_mass_q, k_mass_xr, k_mass_beta, k_mass_d.  The vector kernels run one
// block per (run of TPB nodes, mapped field blockIdx.y): on the small grids of the consistent
// mapping the fields would otherwise be serial work of one thread per node.  Each (block, field)
// partial is the same sum over the same nodes in the same tree order as one slot of a block
// reduction over all fields.

// q = M d on heavy rows (d is 0 on the other nodes); partial (d.q) in slot c
template <int DIM, int R>
__global__ void __launch_bounds__(TPB) k_mass_q(Batch B) {
    PROB_PROLOGUE
    constexpr int SW = 2 * R + 1;
    constexpr int S = DIM == 2 ? SW * SW : SW * SW * SW;
    const int c = blockIdx.y;
    const int64_t N = d->Nnode;
    if (!d->cons || mglob(d)[MG_ALLDONE] != 0.0 || c >= d->ncol) return;   // uniform over the block
    double v = 0.0;
    if (tid < N && d->mheavy[tid]) {
        int n[3];
        node_coords(d, tid, n);
        double q = 0.0;
        for (int e = 0; e < S; ++e) {
            const int64_t k = stencil_nbr<DIM, R>(d, n, e);
            if (k >= 0) q += d->mrow[e * N + tid] * d->md[c * N + k];
        }
        d->mq[c * N + tid] = q;
        v = d->md[c * N + tid] * q;
    }
    double out[1];
    block_sum<1>(&v, out);
    if (threadIdx.x == 0) d->mpart[lb * 3 * MCOL + c] = out[0];
}

// alpha = (r.z) / (d.q) of field c, formed by every block from k_mass_q's partials (the same sum
// in the same order in each), then x += alpha d, r -= alpha q, z = r / M_lumped on heavy rows;
// partials (r.z, r.r) in slots MCOL + 2c, MCOL + 2c + 1, past the (d.q) ones that other blocks
// may still be reading
__global__ void __launch_bounds__(TPB) k_mass_xr(Batch B) {
    PROB_PROLOGUE
    const int c = blockIdx.y;
    const int64_t N = d->Nnode;
    if (!d->cons || mglob(d)[MG_ALLDONE] != 0.0 || c >= d->ncol) return;   // uniform over the block
    __shared__ double alpha;
    {
        double s[1];
        sum_slots<1>(d, node_blocks(d), c, s);
        if (threadIdx.x == 0) {
            const double* m = mcol(d, c);
            alpha = (m[MS_DONE] != 0.0 || s[0] == 0.0) ? 0.0 : m[MS_RZ] / s[0];
        }
        __syncthreads();
    }
    double v[2] = {0.0, 0.0};
    if (tid < N && d->mheavy[tid]) {
        int n[3];
        node_coords(d, tid, n);
        const double m = d->M[pad_index(d, n[0], n[1], n[2])];
        const int64_t k = c * N + tid;
        d->mx[k] += alpha * d->md[k];
        const double r = d->mr[k] - alpha * d->mq[k];
        const double z = r / m;
        d->mr[k] = r;
        d->mz[k] = z;
        v[0] = r * z;
        v[1] = r * r;
    }
    double out[2];
    block_sum<2>(v, out);
    if (threadIdx.x == 0) {
        d->mpart[lb * 3 * MCOL + MCOL + 2 * c] = out[0];
        d->mpart[lb * 3 * MCOL + MCOL + 2 * c + 1] = out[1];
    }
}

__global__ void k_mass_beta(Batch B) {
    const Dev* d = B.d[blockIdx.x];
    if (!d->cons || mglob(d)[MG_ALLDONE] != 0.0) return;
    double s[2 * MCOL];
    sum_slots<2 * MCOL>(d, node_blocks(d), MCOL, s);   // (r.z, r.r) of every field
    if (threadIdx.x == 0) {
        bool all = true;
        for (int c = 0; c < d->ncol; ++c) {
            double* m = mcol(d, c);
            const double rz = s[2 * c], rr = s[2 * c + 1];
            if (m[MS_DONE] == 0.0) {
                m[MS_RR] = rr;
                if (!(rr == rr) || rr <= m[MS_TOL2]) m[MS_DONE] = 1.0;   // NaN also ends (host reports it)
                m[MS_BETA] = (m[MS_DONE] != 0.0 || m[MS_RZ] == 0.0) ? 0.0 : rz / m[MS_RZ];
                m[MS_RZ] = rz;
            } else {
                m[MS_BETA] = 0.0;
            }
            all = all && m[MS_DONE] != 0.0;
        }
        mglob(d)[MG_ALLDONE] = all ? 1.0 : 0.0;
        mglob(d)[MG_ITERS] += 1.0;
    }
}

__global__ void __launch_bounds__(TPB) k_mass_d(Batch B) {
    PROB_PROLOGUE
    const int c = blockIdx.y;
    const int64_t N = d->Nnode;
    if (tid >= N || !d->cons || c >= d->ncol || !d->mheavy[tid]) return;
    const double* m = mcol(d, c);
    if (m[MS_DONE] != 0.0) return;   // converged field: alpha stays 0
    const int64_t k = c * N + tid;
    d->md[k] = d->mz[k] + m[MS_BETA] * d->md[k];
}

// mapped fields back into the nodal arrays; constrained velocity / acceleration components start
// from rest; the Newton start of the free pressure dofs follows the new p
template <int DIM>
__global__ void __launch_bounds__(TPB) k_mass_finish(Batch B) {
    PROB_PROLOGUE
    const int64_t N = d->Nnode;
    if (tid >= N || !d->cons) return;
    int n[3];
    node_coords(d, tid, n);
    const int64_t pn = pad_index(d, n[0], n[1], n[2]);
    if (!(d->M[pn] > 0.0)) return;
    const int bs = DIM + 1;
    const double p = d->mx[tid];
    d->Pn[pn] = p;
    if (!d->bcfix[pn * bs + DIM]) d->X[pn * bs + DIM] = p;
    if (d->dyn) {
        for (int a = 0; a < DIM; ++a) {
            const bool fx = d->bcfix[pn * bs + a] != 0;
            d->vn[pn * 3 + a] = fx ? 0.0 : d->mx[(1 + a) * N + tid];
            d->an[pn * 3 + a] = fx ? 0.0 : d->mx[(1 + DIM + a) * N + tid];
        }
        d->pdn[pn] = d->mx[(1 + 2 * DIM) * N + tid];
        d->pddn[pn] = d->mx[(2 + 2 * DIM) * N + tid];
    }
}

// ---------------------------------------------------------------------------------------------
// point tractions
// ---------------------------------------------------------------------------------------------
// Nodal forces of the point tractions, gathered per node: the points of the buckets whose windows
// can reach the node are visited in bucket order and, inside a bucket, in the sort's id order, so
// every node's sum is formed in the same order on every run (no floating-point atomics).  Along a
// loaded point's normal its face x + lp n takes the grid's linear hat (two nodes: inside the
// point's GIMP window, or within one cell of an original-MPM point's own), along the other axes
// the point's own basis; buckets n - 2 .. n + 1 per axis cover both.
template <int DIM, int SHAPE>
__global__ void __launch_bounds__(TPB) k_point_force(Batch B, const double* __restrict__ F,
                                                     const double* __restrict__ nrm) {
    PROB_PROLOGUE
    if (tid >= d->Nnode) return;
    constexpr int WB = SHAPE ? 3 : 2;
    int n[3];
    node_coords(d, tid, n);
    int clo[3] = {0, 0, 0}, chi[3] = {0, 0, 0};
    for (int a = 0; a < DIM; ++a) {
        clo[a] = n[a] - 2 < 0 ? 0 : n[a] - 2;
        chi[a] = n[a] + 1 > d->nc[a] - 1 ? d->nc[a] - 1 : n[a] + 1;
    }
    const double* P = d->pw;
    const int64_t s = d->ps;
    double acc[DIM];
    for (int a = 0; a < DIM; ++a) acc[a] = 0.0;
    bool hit = false;
    for (int cz = (DIM == 3 ? clo[2] : 0); cz <= (DIM == 3 ? chi[2] : 0); ++cz)
        for (int cy = clo[1]; cy <= chi[1]; ++cy)
            for (int cx = clo[0]; cx <= chi[0]; ++cx) {
                const int64_t c = cx + (int64_t)d->nc[0] * (cy + (int64_t)d->nc[1] * cz);
                const int p0 = d->cstart[c], p1 = d->cstart[c + 1];
                for (int i = p0; i < p1; ++i) {
                    const int64_t id = d->idw[i];
                    double f[DIM];
                    bool any = false;
                    for (int a = 0; a < DIM; ++a) {
                        f[a] = F[id * DIM + a];
                        any |= f[a] != 0.0;
                    }
                    if (!any) continue;
                    double sw = 1.0;
                    bool in = true;
                    for (int a = 0; a < DIM && in; ++a) {
                        double w[3], dw[3], s0v[3];
                        const double xa = P[(PX + a) * s + i], lpa = P[(PLP + a) * s + i];
                        const double na = nrm ? nrm[id * DIM + a] : 0.0;
                        int base, cnt;
                        if (fabs(na) > 0.5) {
                            base = basis_1d<0>(xa + lpa * (na > 0 ? 1.0 : -1.0), 0.0, d->x0[a], d->h, d->nc[a], w, dw, s0v);
                            cnt = 2;
                        } else {
                            base = basis_1d<SHAPE>(xa, lpa, d->x0[a], d->h, d->nc[a], w, dw, s0v);
                            cnt = WB;
                        }
                        const int li = n[a] - base;
                        if (li < 0 || li >= cnt) in = false;
                        else sw *= w[li];
                    }
                    if (!in || sw == 0.0) continue;
                    for (int a = 0; a < DIM; ++a) acc[a] += sw * f[a];
                    hit = true;
                }
            }
    if (!hit) return;
    const int64_t pn = pad_index(d, n[0], n[1], n[2]);
    const int bs = DIM + 1;
    for (int a = 0; a < DIM; ++a) d->fext[pn * bs + a] += acc[a];
}

// ---------------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------------
void launch_point_force(const Group& g, const std::vector<const double*>& F, const std::vector<const double*>& nrm,
                        hipStream_t st) {
    for (size_t q = 0; q < g.ddev.size(); ++q) {
        if (!F[q]) continue;
        Batch B = make_batch({g.ddev[q]}, {g.nnode[q]}, TPB);
        const dim3 gr(B.pfx[B.n]), tb(TPB);
        if (g.dim == 2 && g.shape == 0) hipLaunchKernelGGL((k_point_force<2, 0>), gr, tb, 0, st, B, F[q], nrm[q]);
        else if (g.dim == 2) hipLaunchKernelGGL((k_point_force<2, 1>), gr, tb, 0, st, B, F[q], nrm[q]);
        else hipLaunchKernelGGL((k_point_force<3, 0>), gr, tb, 0, st, B, F[q], nrm[q]);
    }
}

template <int DIM, int SHAPE>
static ppmpm_status mass_solve_t(const Group& g, const std::vector<const Dev*>& hc, hipStream_t st, int* iters) {
    constexpr int R = SHAPE ? 2 : 1;
    Batch Bn = make_batch(g.ddev, g.nnode, TPB);
    Batch B1 = make_batch_one_block(g.ddev);
    const dim3 gn(Bn.pfx[Bn.n]), g1(B1.n), tb(TPB);
    hipLaunchKernelGGL((k_mass_rows<DIM, SHAPE>), gn, tb, 0, st, Bn);
    hipLaunchKernelGGL(k_mass_clear, g1, tb, 0, st, B1);
    hipLaunchKernelGGL(k_mass_max, gn, tb, 0, st, Bn);
    hipLaunchKernelGGL(k_mass_init, gn, tb, 0, st, Bn);
    hipLaunchKernelGGL((k_mass_r0<DIM, R>), gn, tb, 0, st, Bn);
    hipLaunchKernelGGL(k_mass_scal0, g1, tb, 0, st, B1);
    int ncol = 1;
    for (auto* h : hc) ncol = std::max(ncol, h->ncol);
    const dim3 gc(Bn.pfx[Bn.n], ncol);
    std::vector<double> flag(hc.size());
    int it = 0;
    bool done = false;
    while (!done) {
        for (int k = 0; k < MASS_CHECK; ++k) {
            hipLaunchKernelGGL((k_mass_q<DIM, R>), gc, tb, 0, st, Bn);
            hipLaunchKernelGGL(k_mass_xr, gc, tb, 0, st, Bn);
            hipLaunchKernelGGL(k_mass_beta, g1, tb, 0, st, B1);
            hipLaunchKernelGGL(k_mass_d, gc, tb, 0, st, Bn);
        }
        it += MASS_CHECK;
        for (size_t q = 0; q < hc.size(); ++q)
            if (hipMemcpyAsync(&flag[q], hc[q]->mscal + MCOL * MS_STRIDE + MG_ALLDONE, sizeof(double),
                               hipMemcpyDeviceToHost, st) != hipSuccess)
                return PPMPM_E_DEVICE;
        if (hipStreamSynchronize(st) != hipSuccess) return PPMPM_E_DEVICE;
        done = true;
        for (size_t q = 0; q < hc.size(); ++q) done = done && (!hc[q]->cons || flag[q] != 0.0);
        if (!done && it >= MASS_MAXIT) return PPMPM_E_NEWTON;
    }
    // every column must have ended on its tolerance (a NaN residual also ends the iteration)
    for (size_t q = 0; q < hc.size(); ++q) {
        if (!hc[q]->cons) continue;
        double sc[MCOL * MS_STRIDE];
        if (hipMemcpyAsync(sc, hc[q]->mscal, sizeof(sc), hipMemcpyDeviceToHost, st) != hipSuccess) return PPMPM_E_DEVICE;
        if (hipStreamSynchronize(st) != hipSuccess) return PPMPM_E_DEVICE;
        for (int c = 0; c < hc[q]->ncol; ++c)
            if (!(sc[c * MS_STRIDE + MS_RR] <= sc[c * MS_STRIDE + MS_TOL2])) return PPMPM_E_NONFINITE;
    }
    hipLaunchKernelGGL((k_mass_finish<DIM>), gn, tb, 0, st, Bn);
    if (iters) *iters = it;
    return PPMPM_OK;
}

ppmpm_status launch_mass_solve(const Group& g, const std::vector<const Dev*>& hc, hipStream_t st, int* iters) {
    if (g.dim == 2 && g.shape == 0) return mass_solve_t<2, 0>(g, hc, st, iters);
    if (g.dim == 2) return mass_solve_t<2, 1>(g, hc, st, iters);
    return mass_solve_t<3, 0>(g, hc, st, iters);
}

}  // namespace ppm
