// Particle-side kernels of one MPM step (Sec. 3.1, Stages 1, 3 and 4):
//   counting sort of the material points into buckets by the first cell of their basis window
//   (the containing cell for original MPM; ties ordered by point id, so the order and every
//   later sum are deterministic), the per-cell segmented reduction of the
//   projection operator for original MPM (eq. projection-operator), lumped P2G as a per-node
//   gather (eq. map-from-particles-to-nodes), and the G2P update with FLIP velocities and the
//   GIMP domain update (Sec. 3.5).
// All kernels are batch kernels: block b belongs to problem q with B.pfx[q] <= b < B.pfx[q+1].
#include "ppmpm_internal.hpp"
#include "launch.hpp"

namespace ppm {

#define PROB_PROLOGUE                                   \
    const int q = batch_find(B, blockIdx.x);            \
    const Dev* __restrict__ d = B.d[q];                 \
    const int64_t lb = blockIdx.x - B.pfx[q];           \
    const int64_t tid = lb * blockDim.x + threadIdx.x;

__device__ __forceinline__ double& PF_(double* base, int64_t stride, int f, int64_t i) {
    return base[(int64_t)f * stride + i];
}

// ---------------------------------------------------------------------------------------------
// particle state I/O
// ---------------------------------------------------------------------------------------------
__global__ void k_set_particles(Batch B, const double* __restrict__ x, const double* __restrict__ vol,
                                const double* __restrict__ mass, const double* __restrict__ lp,
                                const double* __restrict__ v0, const double* __restrict__ p0) {
    PROB_PROLOGUE
    if (tid >= d->Np) return;
    const int D = d->dim;
    double* P = d->pc;
    const int64_t s = d->ps;
    for (int f = 0; f < NPF; ++f) PF_(P, s, f, tid) = 0.0;
    bool out = false;
    for (int a = 0; a < D; ++a) {
        double xa = x[tid * D + a];
        PF_(P, s, PX + a, tid) = xa;
        if (!(xa >= d->x0[a] && xa <= d->hi[a])) out = true;
        double l = lp ? lp[tid * D + a] : 0.25 * d->h;
        PF_(P, s, PLP + a, tid) = l;
        PF_(P, s, PLP0 + a, tid) = l;
        if (d->shape == 1 && !(l > 0.0 && l <= 0.5 * d->h)) out = true;
        PF_(P, s, PVEL + a, tid) = v0 ? v0[tid * D + a] : 0.0;
        PF_(P, s, PF + a * D + a, tid) = 1.0;
    }
    PF_(P, s, PV, tid) = vol[tid];
    PF_(P, s, PM, tid) = mass[tid];
    PF_(P, s, PP, tid) = p0 ? p0[tid] : 0.0;
    d->idc[tid] = (int)tid;
    if (out) atomicOr(&d->flags[FL_OUTSIDE], 1);
}

// out[i*ncomp + c] in the caller's order from the committed (sorted) state
__global__ void k_get_field(Batch B, int field, int ncomp, double* __restrict__ out) {
    PROB_PROLOGUE
    if (tid >= d->Np) return;
    const int D = d->dim;
    const double* P = d->pc;
    const int64_t s = d->ps;
    const int64_t dst = d->idc[tid];
    if (dst < 0 || dst >= d->Np) { atomicOr(&d->flags[FL_BOUNDS], 1); return; }
    switch (field) {
        case 0: for (int a = 0; a < D; ++a) out[dst * D + a] = P[(PX + a) * s + tid]; break;
        case 1: for (int a = 0; a < D; ++a) out[dst * D + a] = P[(PU + a) * s + tid]; break;
        case 2: out[dst] = P[PP * s + tid]; break;
        case 3: for (int a = 0; a < D * D; ++a) out[dst * D * D + a] = P[(PF + a) * s + tid]; break;
        case 4: out[dst] = P[PV * s + tid]; break;
        case 5: {
            // full 3x3 from xx yy zz xy yz xz
            double sg[6];
            for (int k = 0; k < 6; ++k) sg[k] = P[(PSIG + k) * s + tid];
            double full[9] = {sg[0], sg[3], sg[5], sg[3], sg[1], sg[4], sg[5], sg[4], sg[2]};
            for (int k = 0; k < 9; ++k) out[dst * 9 + k] = full[k];
            break;
        }
        case 6: for (int a = 0; a < D; ++a) out[dst * D + a] = P[(PVEL + a) * s + tid]; break;
        case 7: for (int a = 0; a < D; ++a) out[dst * D + a] = P[(PACC + a) * s + tid]; break;
        case 8: out[dst] = P[PPD * s + tid]; break;
        case 9: out[dst] = P[PPDD * s + tid]; break;
        case 10: for (int a = 0; a < D; ++a) out[dst * D + a] = P[(PLP + a) * s + tid]; break;
        default: break;
    }
}

// ---------------------------------------------------------------------------------------------
// counting sort into window-base buckets
// ---------------------------------------------------------------------------------------------
__global__ void k_zero_counts(Batch B) {
    PROB_PROLOGUE
    if (tid <= d->Ncell) d->ccount[tid] = 0;
}

__global__ void k_sort_keys(Batch B) {
    PROB_PROLOGUE
    if (tid >= d->Np) return;
    const double* P = d->pc;
    const int64_t s = d->ps;
    int64_t cid = 0, mul = 1;
    bool out = false;
    for (int a = 0; a < d->dim; ++a) {
        double xa = P[(PX + a) * s + tid];
        if (!(xa >= d->x0[a] && xa <= d->hi[a])) out = true;
        // bucket = basis window base (the containing cell for original MPM)
        int c = d->shape ? window_base<1>(xa, P[(PLP + a) * s + tid], d->x0[a], d->h, d->nc[a])
                         : window_base<0>(xa, 0.0, d->x0[a], d->h, d->nc[a]);
        cid += c * mul;
        mul *= d->nc[a];
    }
    if (out) atomicOr(&d->flags[FL_OUTSIDE], 1);
    d->key[tid] = (int)cid;
    d->slot[tid] = atomicAdd(&d->ccount[cid], 1);
}

// Exclusive scan of the cell counts: one 1024-thread block per problem over chunks of 4096
// counts, four consecutive counts per thread, a shuffle scan per wavefront and one over the
// sixteen wavefront totals (two barriers per chunk).
__global__ void __launch_bounds__(1024) k_scan_cells(Batch B) {
    const int q = blockIdx.x;
    const Dev* d = B.d[q];
    constexpr int NW = 1024 / 64;
    __shared__ int wsum[NW];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t n = d->Ncell;
    int carry = 0;   // same value in every thread
    for (int64_t base = 0; base < n; base += 4096) {
        const int64_t i0 = base + 4 * (int64_t)threadIdx.x;
        int v[4], incl[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = i0 + k < n ? d->ccount[i0 + k] : 0;
        incl[0] = v[0];
#pragma unroll
        for (int k = 1; k < 4; ++k) incl[k] = incl[k - 1] + v[k];
        int x = incl[3];   // inclusive scan of the thread totals within the wavefront
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(x, off);
            if (lane >= off) x += t;
        }
        if (lane == 63) wsum[wid] = x;
        __syncthreads();
        int wpre = 0, total = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int ws = wsum[w];
            wpre += w < wid ? ws : 0;
            total += ws;
        }
        const int before = carry + wpre + (x - incl[3]);
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (i0 + k < n) d->cstart[i0 + k] = before + incl[k] - v[k];
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) d->cstart[n] = carry;
}

__global__ void k_scatter(Batch B) {
    PROB_PROLOGUE
    if (tid >= d->Np) return;
    int64_t pos = (int64_t)d->cstart[d->key[tid]] + d->slot[tid];
    if (pos < 0 || pos >= d->Np) { atomicOr(&d->flags[FL_BOUNDS], 1); return; }
    d->order[pos] = (int)tid;
}

// Within each cell, order the points by their persistent id (insertion sort; cells are small).
__global__ void k_cell_sort(Batch B) {
    PROB_PROLOGUE
    if (tid >= d->Ncell) return;
    int s0 = d->cstart[tid], s1 = d->cstart[tid + 1];
    int* o = d->order;
    const int* id = d->idc;
    for (int i = s0 + 1; i < s1; ++i) {
        int v = o[i];
        int key = id[v];
        int j = i - 1;
        while (j >= s0 && id[o[j]] > key) {
            o[j + 1] = o[j];
            --j;
        }
        o[j + 1] = v;
    }
}

// Gather the committed state into the working buffer in cell order.
__global__ void k_permute(Batch B) {
    PROB_PROLOGUE
    if (tid >= d->Np) return;
    const int64_t src = d->order[tid];
    const int64_t s = d->ps;
    const double* __restrict__ A = d->pc;
    double* __restrict__ W = d->pw;
    for (int f = 0; f < NPF; ++f) W[f * s + tid] = A[f * s + src];
    d->idw[tid] = d->idc[src];
}

// ---------------------------------------------------------------------------------------------
// projection operator of original MPM: per-cell segmented reduction over the sorted points
// ---------------------------------------------------------------------------------------------
template <int DIM>
__global__ void k_cell_proj(Batch B) {
    PROB_PROLOGUE
    if (tid >= d->Ncell) return;
    constexpr int NV = 1 << DIM;
    int s0 = d->cstart[tid], s1 = d->cstart[tid + 1];
    const double* P = d->pw;
    const int64_t s = d->ps;
    double Ve = 0.0, qv[NV];
    for (int k = 0; k < NV; ++k) qv[k] = 0.0;
    for (int i = s0; i < s1; ++i) {
        double w[DIM][2], dw[2], s0v[2];
        for (int a = 0; a < DIM; ++a)
            basis_1d<0>(P[(PX + a) * s + i], 0.0, d->x0[a], d->h, d->nc[a], w[a], dw, s0v);
        double V = P[PV * s + i];
        Ve += V;
        for (int k = 0; k < NV; ++k) {
            double wk = 1.0;
            for (int a = 0; a < DIM; ++a) wk *= w[a][(k >> a) & 1];
            qv[k] += V * wk;
        }
    }
    for (int k = 0; k < NV; ++k) d->cellpi[tid * NV + k] = Ve > 0.0 ? qv[k] / Ve : 0.0;
}

// ---------------------------------------------------------------------------------------------
// BC arrays (natural node order) -> padded per-dof arrays
// ---------------------------------------------------------------------------------------------
__global__ void k_bc_scatter(Batch B, const uint8_t* __restrict__ ufix, const double* __restrict__ uinc,
                             const uint8_t* __restrict__ pfix, const double* __restrict__ pval,
                             const double* __restrict__ fext, const double* __restrict__ qext) {
    PROB_PROLOGUE
    if (tid >= d->Nnode) return;
    const int D = d->dim, bs = d->b;
    int ix = (int)(tid % d->nn[0]);
    int iy = (int)((tid / d->nn[0]) % d->nn[1]);
    int iz = D == 3 ? (int)(tid / ((int64_t)d->nn[0] * d->nn[1])) : 0;
    int64_t pn = pad_index(d, ix, iy, iz);
    for (int a = 0; a < D; ++a) {
        d->bcfix[pn * bs + a] = ufix ? ufix[tid * D + a] : 0;
        d->bcval[pn * bs + a] = uinc ? uinc[tid * D + a] : 0.0;
        d->fext[pn * bs + a] = fext ? fext[tid * D + a] : 0.0;
    }
    d->bcfix[pn * bs + D] = pfix ? pfix[tid] : 0;
    d->bcval[pn * bs + D] = pval ? pval[tid] : 0.0;
    d->fext[pn * bs + D] = qext ? -qext[tid] : 0.0;
}

// ---------------------------------------------------------------------------------------------
// Stage 1: lumped P2G as a per-node gather, plus dof masks and the Newton start
// ---------------------------------------------------------------------------------------------
template <int DIM, int SHAPE>
__global__ void k_p2g(Batch B) {
    PROB_PROLOGUE
    if (tid >= d->Nnode) return;
    constexpr int WB = SHAPE ? 3 : 2;
    const int bs = DIM + 1;
    int n[3];
    n[0] = (int)(tid % d->nn[0]);
    n[1] = (int)((tid / d->nn[0]) % d->nn[1]);
    n[2] = DIM == 3 ? (int)(tid / ((int64_t)d->nn[0] * d->nn[1])) : 0;
    const int64_t pn = pad_index(d, n[0], n[1], n[2]);
    const double* P = d->pw;
    const int64_t s = d->ps;
    const bool dyn = d->dyn;
    int clo[3] = {0, 0, 0}, chi[3] = {0, 0, 0};
    for (int a = 0; a < DIM; ++a) {
        clo[a] = n[a] - (SHAPE ? 2 : 1);
        chi[a] = n[a] + (SHAPE ? 1 : 0);
        clo[a] = clo[a] < 0 ? 0 : clo[a];
        chi[a] = chi[a] > d->nc[a] - 1 ? d->nc[a] - 1 : chi[a];
    }
    double M = 0, Mp = 0, Vs = 0, Mv[3] = {0, 0, 0}, Ma[3] = {0, 0, 0}, Mpd = 0, Mpdd = 0;
    for (int cz = (DIM == 3 ? clo[2] : 0); cz <= (DIM == 3 ? chi[2] : 0); ++cz)
        for (int cy = clo[1]; cy <= chi[1]; ++cy) {
            int64_t row = (int64_t)d->nc[0] * (cy + (int64_t)d->nc[1] * cz);
            int i0 = d->cstart[row + clo[0]], i1 = d->cstart[row + chi[0] + 1];
            for (int i = i0; i < i1; ++i) {
                double wgt = 1.0;
                bool in = true;
                for (int a = 0; a < DIM; ++a) {
                    double w[3], dw[3], s0v[3];
                    int base = basis_1d<SHAPE>(P[(PX + a) * s + i], P[(PLP + a) * s + i], d->x0[a], d->h,
                                               d->nc[a], w, dw, s0v);
                    int li = n[a] - base;
                    if (li < 0 || li >= WB) { in = false; break; }
                    wgt *= w[li];
                }
                if (!in) continue;
                double m = P[PM * s + i];
                double wm = wgt * m;
                M += wm;
                Mp += wm * P[PP * s + i];
                Vs += wgt * P[PV * s + i];
                if (dyn) {
                    for (int a = 0; a < DIM; ++a) {
                        Mv[a] += wm * P[(PVEL + a) * s + i];
                        Ma[a] += wm * P[(PACC + a) * s + i];
                    }
                    Mpd += wm * P[PPD * s + i];
                    Mpdd += wm * P[PPDD * s + i];
                }
            }
        }
    const bool act = M > 0.0;
    const double inv = act ? 1.0 / M : 0.0;
    d->M[pn] = M;
    d->Pn[pn] = Mp * inv;
    d->Mp[pn] = Vs;
    if (d->cons) {
        // right-hand sides sum S m f of the consistent mapping (kern_mass.hip), natural node order
        const int64_t N = d->Nnode;
        d->mb[tid] = Mp;
        if (dyn) {
            for (int a = 0; a < DIM; ++a) {
                d->mb[(1 + a) * N + tid] = Mv[a];
                d->mb[(1 + DIM + a) * N + tid] = Ma[a];
            }
            d->mb[(1 + 2 * DIM) * N + tid] = Mpd;
            d->mb[(2 + 2 * DIM) * N + tid] = Mpdd;
        }
    }
    if (dyn) {
        for (int a = 0; a < DIM; ++a) {
            bool fx = d->bcfix[pn * bs + a] != 0;
            d->vn[pn * 3 + a] = fx ? 0.0 : Mv[a] * inv;
            d->an[pn * 3 + a] = fx ? 0.0 : Ma[a] * inv;
        }
        d->pdn[pn] = Mpd * inv;
        d->pddn[pn] = Mpdd * inv;
    }
    for (int c = 0; c < bs; ++c) {
        bool fx = d->bcfix[pn * bs + c] != 0;
        d->dfree[pn * bs + c] = (act && !fx) ? 1 : 0;
        double x0v;
        if (!act) x0v = 0.0;
        else if (fx) x0v = d->bcval[pn * bs + c];
        else x0v = (c == DIM) ? Mp * inv : 0.0;
        d->X[pn * bs + c] = x0v;
    }
}

// Largest nodal mass of the step (non-negative doubles order like their bit patterns), then the
// nodes below the negligible-mass fraction of it leave the material: mass, mapped fields, dof masks and the
// Newton start are cleared as for a node without points.
__global__ void k_clear_mmax(Batch B) {
    if (threadIdx.x == 0) B.d[blockIdx.x]->scal[SC_MMAX] = 0.0;
}

__global__ void __launch_bounds__(TPB) k_node_mass_max(Batch B) {
    PROB_PROLOGUE
    double m = 0.0;
    if (tid < d->Nnode) {
        int n[3];
        n[0] = (int)(tid % d->nn[0]);
        n[1] = (int)((tid / d->nn[0]) % d->nn[1]);
        n[2] = d->dim == 3 ? (int)(tid / ((int64_t)d->nn[0] * d->nn[1])) : 0;
        m = d->M[pad_index(d, n[0], n[1], n[2])];
    }
    block_max_nonneg(d->scal + SC_MMAX, m);
}

template <int DIM>
__global__ void k_cut_light_nodes(Batch B) {
    PROB_PROLOGUE
    if (tid >= d->Nnode) return;
    int n[3];
    n[0] = (int)(tid % d->nn[0]);
    n[1] = (int)((tid / d->nn[0]) % d->nn[1]);
    n[2] = DIM == 3 ? (int)(tid / ((int64_t)d->nn[0] * d->nn[1])) : 0;
    const int64_t pn = pad_index(d, n[0], n[1], n[2]);
    const double m = d->M[pn];
    if (!(m > 0.0) || m > d->negl * d->scal[SC_MMAX]) return;
    d->M[pn] = d->Pn[pn] = d->Mp[pn] = d->pdn[pn] = d->pddn[pn] = 0.0;
    for (int a = 0; a < 3; ++a) d->vn[pn * 3 + a] = d->an[pn * 3 + a] = 0.0;
    for (int c = 0; c <= DIM; ++c) {
        d->dfree[pn * (DIM + 1) + c] = 0;
        d->X[pn * (DIM + 1) + c] = 0.0;
    }
}

// Pressure conditions carried by material points (Sec. 5.4): every active node in the basis of a
// flagged point holds the point's value (nodes shared by flagged points with different values
// get one of them).
template <int DIM, int SHAPE>
__global__ void k_point_pfix(Batch B, const uint8_t* __restrict__ flag, const double* __restrict__ val) {
    PROB_PROLOGUE
    if (tid >= d->Np) return;
    const int64_t id = d->idw[tid];
    if (!flag[id]) return;
    constexpr int WB = SHAPE ? 3 : 2;
    const double v = val ? val[id] : 0.0;
    const double* P = d->pw;
    const int64_t s = d->ps;
    double w[DIM][3], dw[3], s0v[3];
    int base[3] = {0, 0, 0};
    for (int a = 0; a < DIM; ++a)
        base[a] = basis_1d<SHAPE>(P[(PX + a) * s + tid], P[(PLP + a) * s + tid], d->x0[a], d->h, d->nc[a], w[a], dw,
                                  s0v);
    for (int k2 = 0; k2 < (DIM == 3 ? WB : 1); ++k2)
        for (int k1 = 0; k1 < WB; ++k1)
            for (int k0 = 0; k0 < WB; ++k0) {
                const int kk[3] = {k0, k1, k2};
                int idx[3] = {0, 0, 0};
                double sw = 1.0;
                bool ok = true;
                for (int a = 0; a < DIM; ++a) {
                    idx[a] = base[a] + kk[a];
                    if (idx[a] < 0 || idx[a] >= d->nn[a]) ok = false;
                    sw *= w[a][kk[a]];
                }
                if (!ok || !(sw > 0.0)) continue;
                const int64_t pn = pad_index(d, idx[0], idx[1], idx[2]);
                if (!(d->M[pn] > 0.0)) continue;
                d->dfree[pn * (DIM + 1) + DIM] = 0;
                d->X[pn * (DIM + 1) + DIM] = v;
            }
}

// Drained free surface (Sec. 5.3): the pore pressure of an active node with an inactive node
// among its 3^dim - 1 neighbours inside the grid is held at zero for the step.  Reads the nodal
// masses of k_p2g, so it runs as a kernel of its own after it.
template <int DIM>
__global__ void k_drain_surface(Batch B) {
    PROB_PROLOGUE
    if (tid >= d->Nnode || !d->drain) return;
    int n[3];
    n[0] = (int)(tid % d->nn[0]);
    n[1] = (int)((tid / d->nn[0]) % d->nn[1]);
    n[2] = DIM == 3 ? (int)(tid / ((int64_t)d->nn[0] * d->nn[1])) : 0;
    const int64_t pn = pad_index(d, n[0], n[1], n[2]);
    if (!(d->M[pn] > 0.0)) return;
    bool surf = false;
    for (int oz = (DIM == 3 ? -1 : 0); oz <= (DIM == 3 ? 1 : 0); ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                const int kx = n[0] + ox, ky = n[1] + oy, kz = n[2] + oz;
                if (kx < 0 || kx >= d->nn[0] || ky < 0 || ky >= d->nn[1]) continue;
                if (DIM == 3 && (kz < 0 || kz >= d->nn[2])) continue;
                surf |= !(d->M[pad_index(d, kx, ky, kz)] > 0.0);
            }
    if (!surf) return;
    const int64_t k = pn * (DIM + 1) + DIM;
    d->dfree[k] = 0;
    d->X[k] = 0.0;
}

// ---------------------------------------------------------------------------------------------
// Stages 3-4: G2P update of the working (sorted) state in place
// ---------------------------------------------------------------------------------------------
template <int DIM, int SHAPE>
__global__ void k_g2p(Batch B) {
    PROB_PROLOGUE
    if (tid >= d->Np) return;
    constexpr int WB = SHAPE ? 3 : 2;
    const int bs = DIM + 1;
    double* P = d->pw;
    const int64_t s = d->ps;
    const int64_t i = tid;
    double w[DIM][3], dw[DIM][3], s0v[DIM][3];
    int base[3] = {0, 0, 0};
    for (int a = 0; a < DIM; ++a)
        base[a] = basis_1d<SHAPE>(P[(PX + a) * s + i], P[(PLP + a) * s + i], d->x0[a], d->h, d->nc[a],
                                  w[a], dw[a], s0v[a]);
    const double dt = d->dt, be = d->beta, ga = d->gamma;
    const bool dyn = d->dyn;
    double dF[DIM * DIM];
    for (int k = 0; k < DIM * DIM; ++k) dF[k] = (k % (DIM + 1) == 0) ? 1.0 : 0.0;
    double du[DIM], pp = 0.0, anp[DIM], acc[DIM], pdq = 0.0, pddq = 0.0;
    for (int a = 0; a < DIM; ++a) du[a] = anp[a] = acc[a] = 0.0;
    constexpr int NN = DIM == 2 ? WB * WB : WB * WB * WB;
    for (int k = 0; k < NN; ++k) {
        int li[3] = {k % WB, (k / WB) % WB, DIM == 3 ? k / (WB * WB) : 0};
        double Sv = 1.0, G[DIM];
        for (int a = 0; a < DIM; ++a) {
            Sv *= w[a][li[a]];
            double gr = 1.0;
            for (int c = 0; c < DIM; ++c) gr *= (c == a) ? dw[c][li[c]] : w[c][li[c]];
            G[a] = gr;
        }
        int64_t pn = pad_index(d, base[0] + li[0], base[1] + li[1], DIM == 3 ? base[2] + li[2] : 0);
        const double* Xn = d->X + pn * bs;
        for (int a = 0; a < DIM; ++a) {
            for (int c = 0; c < DIM; ++c) dF[a * DIM + c] += Xn[a] * G[c];
            du[a] += Sv * Xn[a];
        }
        pp += Sv * Xn[DIM];
        if (dyn) {
            for (int a = 0; a < DIM; ++a) {
                double v0 = d->vn[pn * 3 + a], a0 = d->an[pn * 3 + a];
                double an1 = Xn[a] / (be * dt * dt) - v0 / (be * dt) + (1.0 - 0.5 / be) * a0;
                anp[a] += Sv * a0;
                acc[a] += Sv * an1;
            }
            double dP = Xn[DIM] - d->Pn[pn];
            double pdi = d->ct * dP + d->hc1 * d->pdn[pn] + d->hc2 * d->pddn[pn];
            double pddi = dP / (be * dt * dt) - d->pdn[pn] / (be * dt) + (1.0 - 0.5 / be) * d->pddn[pn];
            pdq += Sv * pdi;
            pddq += Sv * pddi;
        }
    }
    double dJ = det<DIM>(dF);
    if (!(dJ > 0.0)) { atomicOr(&d->flags[FL_INVERTED], 1); return; }
    double Fn[DIM * DIM], F[DIM * DIM];
    for (int k = 0; k < DIM * DIM; ++k) Fn[k] = P[(PF + k) * s + i];
    for (int a = 0; a < DIM; ++a)
        for (int c = 0; c < DIM; ++c) {
            double acc2 = 0.0;
            for (int k = 0; k < DIM; ++k) acc2 += dF[a * DIM + k] * Fn[k * DIM + c];
            F[a * DIM + c] = acc2;
        }
    for (int k = 0; k < DIM * DIM; ++k) P[(PF + k) * s + i] = F[k];
    P[PV * s + i] *= dJ;
    bool out = false;
    for (int a = 0; a < DIM; ++a) {
        P[(PU + a) * s + i] += du[a];
        double xn = P[(PX + a) * s + i] + du[a];
        P[(PX + a) * s + i] = xn;
        if (!(xn >= d->x0[a] && xn <= d->hi[a])) out = true;
    }
    if (out) atomicOr(&d->flags[FL_OUTSIDE], 1);
    P[PP * s + i] = pp;
    if (dyn) {
        for (int a = 0; a < DIM; ++a) {
            P[(PVEL + a) * s + i] += dt * ((1.0 - ga) * anp[a] + ga * acc[a]);
            P[(PACC + a) * s + i] = acc[a];
        }
        P[PPD * s + i] = pdq;
        P[PPDD * s + i] = pddq;
    }
    double tau[DIM * DIM], tzz;
    kirchhoff_tangent<DIM>(d->model, d->lam, d->G, F, tau, &tzz, nullptr);
    double J = det<DIM>(F);
    if (DIM == 2) {
        P[(PSIG + 0) * s + i] = tau[0] / J;
        P[(PSIG + 1) * s + i] = tau[3] / J;
        P[(PSIG + 2) * s + i] = tzz / J;
        P[(PSIG + 3) * s + i] = tau[1] / J;
        P[(PSIG + 4) * s + i] = 0.0;
        P[(PSIG + 5) * s + i] = 0.0;
    } else {
        P[(PSIG + 0) * s + i] = tau[0] / J;
        P[(PSIG + 1) * s + i] = tau[4] / J;
        P[(PSIG + 2) * s + i] = tau[8] / J;
        P[(PSIG + 3) * s + i] = tau[1] / J;
        P[(PSIG + 4) * s + i] = tau[5] / J;
        P[(PSIG + 5) * s + i] = tau[2] / J;
    }
    if (SHAPE == 1 && DIM == 2) {
        // right stretch U = (C + sqrt(det C) 1) / sqrt(tr C + 2 sqrt(det C)), C = F^T F
        double C00 = F[0] * F[0] + F[2] * F[2], C01 = F[0] * F[1] + F[2] * F[3], C11 = F[1] * F[1] + F[3] * F[3];
        double sd = sqrt(C00 * C11 - C01 * C01);
        double nrm = 1.0 / sqrt(C00 + C11 + 2.0 * sd);
        double U00 = (C00 + sd) * nrm, U11 = (C11 + sd) * nrm;
        double l0 = P[(PLP0 + 0) * s + i] * U00, l1 = P[(PLP0 + 1) * s + i] * U11;
        P[(PLP + 0) * s + i] = fmin(l0, 0.5 * d->h);
        P[(PLP + 1) * s + i] = fmin(l1, 0.5 * d->h);
    }
}

// ---------------------------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------------------------
void launch_set_particles(const Dev* dd, int64_t np, const double* x, const double* vol, const double* mass,
                          const double* lp, const double* v0, const double* p0, hipStream_t st) {
    Batch B = make_batch({dd}, {np}, TPB);
    hipLaunchKernelGGL(k_set_particles, dim3(B.pfx[B.n]), dim3(TPB), 0, st, B, x, vol, mass, lp, v0, p0);
}

void launch_get_field(const Dev* dd, int64_t np, int field, int ncomp, double* out, hipStream_t st) {
    Batch B = make_batch({dd}, {np}, TPB);
    hipLaunchKernelGGL(k_get_field, dim3(B.pfx[B.n]), dim3(TPB), 0, st, B, field, ncomp, out);
}

void launch_sort(const Group& g, hipStream_t st) {
    Batch Bc = make_batch(g.ddev, g.ncell1, TPB);
    hipLaunchKernelGGL(k_zero_counts, dim3(Bc.pfx[Bc.n]), dim3(TPB), 0, st, Bc);
    Batch Bp = make_batch(g.ddev, g.np, TPB);
    hipLaunchKernelGGL(k_sort_keys, dim3(Bp.pfx[Bp.n]), dim3(TPB), 0, st, Bp);
    Batch Bs = make_batch_one_block(g.ddev);
    hipLaunchKernelGGL(k_scan_cells, dim3(Bs.n), dim3(1024), 0, st, Bs);
    hipLaunchKernelGGL(k_scatter, dim3(Bp.pfx[Bp.n]), dim3(TPB), 0, st, Bp);
    Batch Bn = make_batch(g.ddev, g.ncell, TPB);
    hipLaunchKernelGGL(k_cell_sort, dim3(Bn.pfx[Bn.n]), dim3(TPB), 0, st, Bn);
    PPM_TIMED(KT_PERMUTE, st, hipLaunchKernelGGL(k_permute, dim3(Bp.pfx[Bp.n]), dim3(TPB), 0, st, Bp));
}

void launch_bc(const Dev* dd, int64_t nnode, const uint8_t* uf, const double* ui, const uint8_t* pf,
               const double* pv, const double* fe, const double* qe, hipStream_t st) {
    Batch B = make_batch({dd}, {nnode}, TPB);
    hipLaunchKernelGGL(k_bc_scatter, dim3(B.pfx[B.n]), dim3(TPB), 0, st, B, uf, ui, pf, pv, fe, qe);
}

void launch_p2g(const Group& g, hipStream_t st) {
    Batch B = make_batch(g.ddev, g.nnode, TPB);
    if (g.dim == 2 && g.shape == 0) PPM_TIMED(KT_P2G, st, hipLaunchKernelGGL((k_p2g<2, 0>), dim3(B.pfx[B.n]), dim3(TPB), 0, st, B));
    else if (g.dim == 2 && g.shape == 1) PPM_TIMED(KT_P2G, st, hipLaunchKernelGGL((k_p2g<2, 1>), dim3(B.pfx[B.n]), dim3(TPB), 0, st, B));
    else PPM_TIMED(KT_P2G, st, hipLaunchKernelGGL((k_p2g<3, 0>), dim3(B.pfx[B.n]), dim3(TPB), 0, st, B));
}

void launch_cut_light_nodes(const Group& g, hipStream_t st) {
    Batch B = make_batch(g.ddev, g.nnode, TPB);
    Batch B1 = make_batch_one_block(g.ddev);
    hipLaunchKernelGGL(k_clear_mmax, dim3(B1.n), dim3(64), 0, st, B1);
    hipLaunchKernelGGL(k_node_mass_max, dim3(B.pfx[B.n]), dim3(TPB), 0, st, B);
    if (g.dim == 2) hipLaunchKernelGGL((k_cut_light_nodes<2>), dim3(B.pfx[B.n]), dim3(TPB), 0, st, B);
    else hipLaunchKernelGGL((k_cut_light_nodes<3>), dim3(B.pfx[B.n]), dim3(TPB), 0, st, B);
}

void launch_point_pfix(const Group& g, const std::vector<const uint8_t*>& flag, const std::vector<const double*>& val,
                       hipStream_t st) {
    for (size_t q = 0; q < g.ddev.size(); ++q) {
        if (!flag[q]) continue;
        Batch B = make_batch({g.ddev[q]}, {g.np[q]}, TPB);
        const dim3 gr(B.pfx[B.n]), tb(TPB);
        if (g.dim == 2 && g.shape == 0) hipLaunchKernelGGL((k_point_pfix<2, 0>), gr, tb, 0, st, B, flag[q], val[q]);
        else if (g.dim == 2) hipLaunchKernelGGL((k_point_pfix<2, 1>), gr, tb, 0, st, B, flag[q], val[q]);
        else hipLaunchKernelGGL((k_point_pfix<3, 0>), gr, tb, 0, st, B, flag[q], val[q]);
    }
}

void launch_drain_surface(const Group& g, hipStream_t st) {
    Batch B = make_batch(g.ddev, g.nnode, TPB);
    if (g.dim == 2) hipLaunchKernelGGL((k_drain_surface<2>), dim3(B.pfx[B.n]), dim3(TPB), 0, st, B);
    else hipLaunchKernelGGL((k_drain_surface<3>), dim3(B.pfx[B.n]), dim3(TPB), 0, st, B);
}

void launch_cell_proj(const Group& g, hipStream_t st) {
    Batch B = make_batch(g.ddev, g.ncell, TPB);
    if (g.dim == 2) hipLaunchKernelGGL((k_cell_proj<2>), dim3(B.pfx[B.n]), dim3(TPB), 0, st, B);
    else hipLaunchKernelGGL((k_cell_proj<3>), dim3(B.pfx[B.n]), dim3(TPB), 0, st, B);
}

void launch_g2p(const Group& g, hipStream_t st) {
    Batch B = make_batch(g.ddev, g.np, TPB);
    if (g.dim == 2 && g.shape == 0) PPM_TIMED(KT_G2P, st, hipLaunchKernelGGL((k_g2p<2, 0>), dim3(B.pfx[B.n]), dim3(TPB), 0, st, B));
    else if (g.dim == 2 && g.shape == 1) PPM_TIMED(KT_G2P, st, hipLaunchKernelGGL((k_g2p<2, 1>), dim3(B.pfx[B.n]), dim3(TPB), 0, st, B));
    else PPM_TIMED(KT_G2P, st, hipLaunchKernelGGL((k_g2p<3, 0>), dim3(B.pfx[B.n]), dim3(TPB), 0, st, B));
}

}  // namespace ppm
