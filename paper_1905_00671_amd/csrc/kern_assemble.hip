// Residual and Jacobian assembly at the material points (Sec. 3.1-3.4, Sec. 4.2).
//
// Two passes per Newton iteration:
//   k_records   one thread per (sorted) material point: basis at x_n, relative deformation
//               dF = 1 + sum U (x) grad_n S, stress, tangent and every per-point coefficient the
//               residual and the Jacobian need (the point's "quadrature record", see RecRef);
//   k_residual  blocks of 64-node tiles (16x4 / 8x8x1), four wavefronts per tile each gathering a
//               quarter of the basis-window buckets: R_i from the points whose basis reaches node i
//               (no atomics, fixed summation order), boundary conditions, per-block partial norms;
//   k_jacobian  one thread per (grid node i, row component, column component), the component
//               pair uniform per block: for each point reaching node i, the entries of all its
//               column blocks J_ik come from one set of record loads; the node's fixed-stencil
//               block row is accumulated in registers and written once (no atomics).
// Points are bucketed by the first cell of their basis window, so the points that see node i at
// window position l are exactly those of bucket i - l: both gathers loop over l at compile time
// and every lane of a wavefront runs the same specialized code.
// Residual terms (current configuration, dv = det(dF) V_n, grad S = dF^{-T} grad_n S; kappa is
// constant or the Kozeny-Carman mobility of the volume ratio det(dF) det(F_n), eq. kozeny-carman):
//   R_mom_i  = -(V_n/J_n) tau' grad S_i + dv p^h grad S_i + m S_i (g - a^h)       eq. residual-momentum
//   R_mass_i = dv S_i theta + dv kappa grad S_i.(grad p^h - rho_f (g - a^h))       eq. residual-mass
//              + tau V_n (S_i - Pi S_i)(pdot^h - Pi pdot^h)                       eq. stab-term-ppp
// theta = ln(dJ)/dt (eq. implicit-euler) or div v^h (eq. newmark); the stabilization integral
// is taken on the t_n configuration so that it is linear in P; Pi is the per-cell particle
// average (original MPM) or the constant GIMP basis S0 (Sec. 4.4).
#include "ppmpm_internal.hpp"
#include "launch.hpp"

namespace ppm {

#define PROB_PROLOGUE                                   \
    const int q = batch_find(B, blockIdx.x);            \
    const Dev* __restrict__ d = B.d[q];                 \
    const int64_t lb = blockIdx.x - B.pfx[q];           \
    const int64_t tid = lb * blockDim.x + threadIdx.x;

// The record of point i, written through rec (global memory, or the wavefront's LDS stage).
template <int DIM, int SHAPE, typename Rec>
__device__ __forceinline__ void record_point(const Dev* __restrict__ d, int64_t i, const Rec& rec) {
    constexpr int WB = SHAPE ? 3 : 2;
    constexpr int NN = DIM == 2 ? WB * WB : WB * WB * WB;
    using L = RecLayout<DIM, WB>;
    const int bs = DIM + 1;
    const double* P = d->pw;
    const int64_t s = d->ps;
    double w[DIM][3], dw[DIM][3], s0v[DIM][3];
    int base[3] = {0, 0, 0};
    for (int a = 0; a < DIM; ++a) {
        base[a] = basis_1d<SHAPE>(P[(PX + a) * s + i], P[(PLP + a) * s + i], d->x0[a], d->h, d->nc[a], w[a],
                                  dw[a], s0v[a]);
        for (int k = 0; k < WB; ++k) {
            rec[L::W_ + a * WB + k] = w[a][k];
            rec[L::DW_ + a * WB + k] = dw[a][k];
            rec[L::S0_ + a * WB + k] = s0v[a][k];
        }
    }
    int64_t cid = 0;
    if (SHAPE == 0) {
        int64_t mul = 1;
        for (int a = 0; a < DIM; ++a) { cid += base[a] * mul; mul *= d->nc[a]; }
    }
    const double dt = d->dt, be = d->beta, ga = d->gamma;
    const bool dyn = d->dyn;
    // pass 1: relative deformation dF = 1 + sum_k U_k (x) grad_n S_k
    double dF[DIM * DIM];
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) dF[k] = (k % (DIM + 1) == 0) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < NN; ++k) {
        const int li[3] = {k % WB, (k / WB) % WB, DIM == 3 ? k / (WB * WB) : 0};
        double G[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            double gr = 1.0;
#pragma unroll
            for (int c = 0; c < DIM; ++c) gr *= (c == a) ? dw[c][li[c]] : w[c][li[c]];
            G[a] = gr;
        }
        const int64_t pn = pad_index(d, base[0] + li[0], base[1] + li[1], DIM == 3 ? base[2] + li[2] : 0);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const double u = d->X[pn * bs + a];
#pragma unroll
            for (int c = 0; c < DIM; ++c) dF[a * DIM + c] += u * G[c];
        }
    }
    double dJ = det<DIM>(dF);
    if (!(dJ > 0.0)) {
        atomicOr(&d->flags[FL_INVERTED], 1);
        dJ = 1.0;
        for (int k = 0; k < DIM * DIM; ++k) dF[k] = (k % (DIM + 1) == 0) ? 1.0 : 0.0;
    }
    double f[DIM * DIM], F[DIM * DIM], detFn;
    inverse<DIM>(dF, f);
    {
        double Fn[DIM * DIM];
#pragma unroll
        for (int k = 0; k < DIM * DIM; ++k) Fn[k] = P[(PF + k) * s + i];
        detFn = det<DIM>(Fn);
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
            for (int c = 0; c < DIM; ++c) {
                double t = 0.0;
#pragma unroll
                for (int k = 0; k < DIM; ++k) t += dF[a * DIM + k] * Fn[k * DIM + c];
                F[a * DIM + c] = t;
            }
    }
    const double Vn = P[PV * s + i], m = P[PM * s + i];
    const double V0 = Vn / detFn;
    const double dv = dJ * Vn;
    // mobility: constant, or Kozeny-Carman in the volume ratio dJ det(F_n)
    double kap = d->kappa, kapj = 0.0;
    if (d->phi0 > 0.0) kozeny_carman(d->kappa, d->phi0, dJ * detFn, &kap, &kapj);
    // pass 2: pressure, its gradient, the stabilization term and (Newmark) a^h, grad v
    double ph = 0.0, gp[DIM], ah[DIM], l[DIM * DIM], pst = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) gp[a] = ah[a] = 0.0;
#pragma unroll
    for (int k = 0; k < DIM * DIM; ++k) l[k] = 0.0;
#pragma unroll
    for (int k = 0; k < NN; ++k) {
        const int li[3] = {k % WB, (k / WB) % WB, DIM == 3 ? k / (WB * WB) : 0};
        double sv = 1.0, s0p = 1.0, G[DIM], gS[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            sv *= w[a][li[a]];
            s0p *= s0v[a][li[a]];
            double gr = 1.0;
#pragma unroll
            for (int c = 0; c < DIM; ++c) gr *= (c == a) ? dw[c][li[c]] : w[c][li[c]];
            G[a] = gr;
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            double t = 0.0;
#pragma unroll
            for (int c = 0; c < DIM; ++c) t += f[c * DIM + a] * G[c];
            gS[a] = t;
        }
        const double Pi = SHAPE ? s0p : d->cellpi[cid * (1 << DIM) + k];
        const int64_t pn = pad_index(d, base[0] + li[0], base[1] + li[1], DIM == 3 ? base[2] + li[2] : 0);
        const double Pk = d->X[pn * bs + DIM];
        double pdot = d->ct * (Pk - d->Pn[pn]);
        ph += sv * Pk;
#pragma unroll
        for (int a = 0; a < DIM; ++a) gp[a] += Pk * gS[a];
        if (dyn) {
            pdot += d->hc1 * d->pdn[pn] + d->hc2 * d->pddn[pn];
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                const double u = d->X[pn * bs + a], v0 = d->vn[pn * 3 + a], a0 = d->an[pn * 3 + a];
                const double acc = u / (be * dt * dt) - v0 / (be * dt) + (1.0 - 0.5 / be) * a0;
                const double vel = ga / (be * dt) * u + (1.0 - ga / be) * v0 + (1.0 - 0.5 * ga / be) * dt * a0;
                ah[a] += sv * acc;
#pragma unroll
                for (int c = 0; c < DIM; ++c) l[a * DIM + c] += vel * gS[c];
            }
        }
        pst += (sv - Pi) * pdot;
    }
    double theta;
    if (dyn) {
        theta = 0.0;
        for (int a = 0; a < DIM; ++a) theta += l[a * DIM + a];
    } else {
        theta = log(dJ) / dt;
    }
    double wv[DIM];
    for (int a = 0; a < DIM; ++a) wv[a] = gp[a] - d->rho_f * (d->g[a] - ah[a]);
    // Kelvin-type viscous stress of the Newmark velocity field, sigma_vis = alpha (lam tr l 1 +
    // G (l + l^T)); its linearization is folded into the 2D tangent below and formed in closed
    // form by the 3D cell-matrix kernel
    const bool vis = dyn && d->alpha_vis != 0.0;
    double svis[DIM * DIM];
    for (int k = 0; k < DIM * DIM; ++k) svis[k] = 0.0;
    if (vis) {
        const double al = d->alpha_vis;
        double tr = 0.0;
        for (int a = 0; a < DIM; ++a) tr += l[a * DIM + a];
        for (int a = 0; a < DIM; ++a)
            for (int c = 0; c < DIM; ++c)
                svis[a * DIM + c] = al * (d->G * (l[a * DIM + c] + l[c * DIM + a]) + (a == c ? d->lam * tr : 0.0));
    }
    // Kirchhoff stress; 2D: the tangent with the geometric, pressure and damping terms folded in,
    // with w_c = gamma/(beta dt) e_c - l e_c the damping terms are
    //   dAbar_{ab,ce} = -dv alpha (lam d_ab w_c^e + G d_be w_c^a + G d_ae w_c^b)
    //                   - dv svis_ab d_ce + dv svis_ae d_bc
    double tau[DIM * DIM], tzz;
    if constexpr (DIM == 2) {
        double T[16];
        kirchhoff_tangent<2>(d->model, d->lam, d->G, F, tau, &tzz, T);
        const double al = d->alpha_vis, vg = ga / (be * dt);
        for (int a = 0; a < DIM; ++a)
            for (int bb = 0; bb < DIM; ++bb)
                for (int c = 0; c < DIM; ++c)
                    for (int e = 0; e < DIM; ++e) {
                        double v = -V0 * T[((a * DIM + bb) * DIM + c) * DIM + e];
                        if (bb == c) v += V0 * tau[a * DIM + e];
                        if (a == bb && c == e) v += dv * ph;
                        if (a == e && bb == c) v -= dv * ph;
                        if (vis) {
                            // w_c^m = vg d_mc - l_mc
                            const double wce = (e == c ? vg : 0.0) - l[e * DIM + c];
                            const double wca = (a == c ? vg : 0.0) - l[a * DIM + c];
                            const double wcb = (bb == c ? vg : 0.0) - l[bb * DIM + c];
                            double t = 0.0;
                            if (a == bb) t += d->lam * wce;
                            if (bb == e) t += d->G * wca;
                            if (a == e) t += d->G * wcb;
                            v -= dv * al * t;
                            if (c == e) v -= dv * svis[a * DIM + bb];
                            if (bb == c) v += dv * svis[a * DIM + e];
                        }
                        rec[L::AB_ + ((a * DIM + bb) * DIM + c) * DIM + e] = v;
                    }
    } else {
        // neo-Hookean (the 3D model): the closed-form coefficients of the displacement block
        kirchhoff_tangent<3>(d->model, d->lam, d->G, F, tau, &tzz, nullptr);
        double bm[9];
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 3; ++c) {
                double t = 0.0;
                for (int k = 0; k < 3; ++k) t += F[a * 3 + k] * F[c * 3 + k];
                bm[a * 3 + c] = t;
            }
        const double lnJ = log(det<3>(F));   // as in the Kirchhoff stress
        rec[L::VG_] = V0 * d->G;
        rec[L::BM_ + 0] = bm[0];
        rec[L::BM_ + 1] = bm[4];
        rec[L::BM_ + 2] = bm[8];
        rec[L::BM_ + 3] = bm[1];
        rec[L::BM_ + 4] = bm[5];
        rec[L::BM_ + 5] = bm[2];
        rec[L::C1_] = V0 * (d->lam * lnJ - d->G) - dv * ph;
        rec[L::C2_] = dv * ph - V0 * d->lam;
        rec[L::SV_ + 0] = svis[0];
        rec[L::SV_ + 1] = svis[4];
        rec[L::SV_ + 2] = svis[8];
        rec[L::SV_ + 3] = svis[1];
        rec[L::SV_ + 4] = svis[5];
        rec[L::SV_ + 5] = svis[2];
    }
    for (int k = 0; k < DIM * DIM; ++k) {
        rec[L::FI_ + k] = f[k];
        rec[L::LV_ + k] = dyn ? dv * l[k] : 0.0;
        int a = k / DIM, c = k % DIM;
        rec[L::SG_ + k] = -V0 * tau[k] + (a == c ? dv * ph : 0.0) - dv * svis[k];
    }
    rec[L::DV_] = dv;
    rec[L::CM_] = dyn ? m / (be * dt * dt) : 0.0;
    rec[L::BV_] = dyn ? dv * (theta + ga / (be * dt)) : dv * (1.0 + log(dJ)) / dt;
    rec[L::DK_] = dv * kap;
    rec[L::KJ_] = dv * kapj;
    for (int a = 0; a < DIM; ++a) {
        rec[L::GP_ + a] = gp[a];
        rec[L::QW_ + a] = wv[a];
        rec[L::BF_ + a] = m * (d->g[a] - ah[a]);
    }
    rec[L::EE_] = dyn ? dv * kap * d->rho_f / (be * dt * dt) : 0.0;
    rec[L::TC_] = d->tau * d->ct * Vn;
    rec[L::DT_] = dv * theta;
    rec[L::ST_] = d->tau * Vn * pst;
}

// A point's record in its wavefront's LDS stage: a row of whole 16-word groups per lane, the word
// index swizzled within its group by the lane (k ^ (lane & 15)) so that the 64 lanes writing the
// same field spread over the banks.
struct StageRec {
    double* b;
    int sw;
    __device__ __forceinline__ double& operator[](int k) const { return b[k ^ sw]; }
};

// One thread per (sorted) material point.  The records are staged in LDS and each wavefront then
// stores its 64 records (a contiguous range) with 16-byte stores that cover whole cache lines;
// written directly, the N stores of a thread land N words apart across the wavefront, and the
// partly written lines left L2 as 1.8x the record bytes (3D: 8.1 GB per launch for 4.5 GB).
// The stage is 160 KB (3D) / 128 KB (2D) per block, one block per CU: the kernel's registers
// allow one wavefront per SIMD anyway.
template <int DIM, int SHAPE>
__global__ void __launch_bounds__(TPB) k_records(Batch B) {
    PROB_PROLOGUE
    using L = RecLayout<DIM, SHAPE ? 3 : 2>;
    constexpr int NW = L::N;                       // words per record
    constexpr int NS = (NW + 15) / 16 * 16;        // stage row
    constexpr int USED = DIM == 3 ? L::S0_ + 6 : NW;   // 3D: two padding words close the record
    __shared__ double stage[(TPB / 64) * 64 * NS];
    const int lane = threadIdx.x & 63;
    double* ws = stage + (threadIdx.x >> 6) * 64 * NS;
    const int64_t p0 = tid - lane;   // first point of the wavefront
    if (p0 >= d->Np) return;         // uniform over the wavefront
    const int nv = (int)min((int64_t)64, d->Np - p0);
    if (lane < nv) {
        const StageRec rec{ws + lane * NS, lane & 15};
#pragma unroll
        for (int k = USED; k < NW; ++k) rec[k] = 0.0;
        record_point<DIM, SHAPE>(d, tid, rec);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double* g = d->rec + p0 * NW;   // 16-byte aligned: p0 is a multiple of 64
    const int total = nv * NW;
#pragma unroll 4
    for (int j = 0; j < (64 * NW + 127) / 128; ++j) {
        const int q = j * 128 + 2 * lane;   // word offset inside the wavefront's records
        if (q >= total) continue;
        const int r0 = q / NW, w0 = q - r0 * NW;
        const double v0 = ws[r0 * NS + (w0 ^ (r0 & 15))];
        if (q + 1 < total) {
            const int r1 = (q + 1) / NW, w1 = q + 1 - r1 * NW;
            double2 v;
            v.x = v0;
            v.y = ws[r1 * NS + (w1 ^ (r1 & 15))];
            *reinterpret_cast<double2*>(g + q) = v;
        } else {
            g[q] = v0;
        }
    }
}

// Node of tile lane t: blocks cover tiles of TILE_X x TILE_Y (x TILE_Z) nodes so that the
// lanes of a wavefront gather from overlapping particle sets.
template <int DIM>
__device__ __forceinline__ bool tile_node(const Dev* d, int64_t tile, int t, int* n, int64_t* row) {
    constexpr int tx = DIM == 2 ? TILE2X : TILE3X, ty = DIM == 2 ? TILE2Y : TILE3Y;
    const int ntx = (d->nn[0] + tx - 1) / tx, nty = (d->nn[1] + ty - 1) / ty;
    const int64_t bx = tile % ntx, by = (tile / ntx) % nty, bz = tile / ((int64_t)ntx * nty);
    n[0] = (int)(bx * tx + t % tx);
    n[1] = (int)(by * ty + (t / tx) % ty);
    n[2] = DIM == 3 ? (int)(bz * TILE3Z + t / (tx * ty)) : 0;
    for (int a = 0; a < DIM; ++a)
        if (n[a] >= d->nn[a]) return false;
    *row = n[0] + (int64_t)d->nn[0] * (n[1] + (int64_t)d->nn[1] * n[2]);
    return true;
}

// Points of the bucket (cell) n - l, l the window-local index LI of node n: exactly the points
// whose basis window places node n at LI.  Returns false when that bucket is off the grid.
template <int DIM, int WB, int LI>
__device__ __forceinline__ bool bucket_of(const Dev* d, const int* n, int64_t* cid, int* p0, int* p1) {
    constexpr int l0 = LI % WB, l1 = (LI / WB) % WB, l2 = DIM == 3 ? LI / (WB * WB) : 0;
    const int c0 = n[0] - l0, c1 = n[1] - l1, c2 = DIM == 3 ? n[2] - l2 : 0;
    if (c0 < 0 || c0 >= d->nc[0] || c1 < 0 || c1 >= d->nc[1]) return false;
    if (DIM == 3 && (c2 < 0 || c2 >= d->nc[2])) return false;
    *cid = c0 + (int64_t)d->nc[0] * (c1 + (int64_t)d->nc[1] * c2);
    *p0 = d->cstart[*cid];
    *p1 = d->cstart[*cid + 1];
    return true;
}

// Residual contributions to node n of the points of bucket n - l (LI = window index of n).
template <int DIM, int SHAPE, int LI>
__device__ __forceinline__ void res_bucket(const Dev* __restrict__ d, const int* n, double* r, int part) {
    constexpr int WB = SHAPE ? 3 : 2;
    constexpr int NN = DIM == 2 ? WB * WB : WB * WB * WB;
    if constexpr (LI < NN) {
      if (LI * RES_PARTS / NN == part) {
        constexpr int li[3] = {LI % WB, (LI / WB) % WB, DIM == 3 ? LI / (WB * WB) : 0};
        using L = RecLayout<DIM, WB>;
        int64_t cid;
        int p0, p1;
        if (!bucket_of<DIM, WB, LI>(d, n, &cid, &p0, &p1)) p0 = p1 = 0, cid = 0;
        // original MPM: Pi S_n of the cell, the same for every point of the bucket
        const double pic = (SHAPE || p1 <= p0) ? 0.0 : d->cellpi[cid * NN + LI];
        for (int p = p0; p < p1; ++p) {
            const RecRef rc(d->rec, p, L::N);
            double w[DIM], dw[DIM], Sv = 1.0, s0 = 1.0;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                w[a] = rc[L::W_ + a * WB + li[a]];
                dw[a] = rc[L::DW_ + a * WB + li[a]];
                if (SHAPE) s0 *= rc[L::S0_ + a * WB + li[a]];
                Sv *= w[a];
            }
            double G[DIM], gS[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                double g = 1.0;
#pragma unroll
                for (int c = 0; c < DIM; ++c) g *= (c == a) ? dw[c] : w[c];
                G[a] = g;
            }
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                double t = 0.0;
#pragma unroll
                for (int c = 0; c < DIM; ++c) t += rc[L::FI_ + c * DIM + a] * G[c];
                gS[a] = t;
            }
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                double t = rc[L::BF_ + a] * Sv;
#pragma unroll
                for (int c = 0; c < DIM; ++c) t += rc[L::SG_ + a * DIM + c] * gS[c];
                r[a] += t;
            }
            const double Pi = SHAPE ? s0 : pic;
            double gw = 0.0;
#pragma unroll
            for (int a = 0; a < DIM; ++a) gw += gS[a] * rc[L::QW_ + a];
            r[DIM] += Sv * rc[L::DT_] + rc[L::DK_] * gw + rc[L::ST_] * (Sv - Pi);
        }
      }
        res_bucket<DIM, SHAPE, LI + 1>(d, n, r, part);
    }
}

// One block per tile of RES_NODES grid nodes, RES_PARTS wavefronts per tile: wavefront j gathers
// the buckets LI with LI * RES_PARTS / NN = j for all nodes of the tile (the gather is latency-bound;
// four times as many wavefronts, each walking a quarter of a node's points), then the parts are
// added in LDS in a fixed order and the first wavefront finishes its nodes.
template <int DIM, int SHAPE>
__global__ void __launch_bounds__(TPB) k_residual(Batch B) {
    static_assert(RES_NODES * RES_PARTS == TPB, "one wavefront per part");
    const int q = batch_find(B, blockIdx.x);
    const Dev* __restrict__ d = B.d[q];
    const int64_t lb = blockIdx.x - B.pfx[q];
    const int bs = DIM + 1;
    const int part = threadIdx.x / RES_NODES, ln = threadIdx.x % RES_NODES;
    __shared__ double sr[RES_PARTS][DIM + 1][RES_NODES];
    double ru2 = 0.0, rp2 = 0.0;
    bool bad = false;
    int n[3];
    int64_t row;
    const bool in = tile_node<DIM>(d, lb, ln, n, &row);
    double r[DIM + 1];
    for (int c = 0; c <= DIM; ++c) r[c] = 0.0;
    if (in) res_bucket<DIM, SHAPE, 0>(d, n, r, part);
    for (int c = 0; c <= DIM; ++c) sr[part][c][ln] = r[c];
    __syncthreads();
    if (part == 0 && in) {
        const int64_t pn = pad_index(d, n[0], n[1], n[2]);
        for (int c = 0; c <= DIM; ++c) {
            double v = 0.0;
#pragma unroll
            for (int j = 0; j < RES_PARTS; ++j) v += sr[j][c][ln];
            v += d->fext[pn * bs + c];
            if (!d->dfree[pn * bs + c]) v = 0.0;
            if (!isfinite(v)) bad = true;
            d->Rv[pn * bs + c] = v;
            if (c < DIM) ru2 += v * v;
            else rp2 += v * v;
        }
    }
    if (bad) atomicOr(&d->flags[FL_NONFINITE], 1);
    // block partial sums (deterministic tree)
    __shared__ double sh[2][TPB];
    sh[0][threadIdx.x] = ru2;
    sh[1][threadIdx.x] = rp2;
    __syncthreads();
    for (int off = TPB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + off];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        d->partial[lb * 4 + 0] = sh[0][0];
        d->partial[lb * 4 + 1] = sh[1][0];
    }
}

// 3D residual in two passes: the points of a cell (its sort bucket) reach exactly the cell's 8
// corner nodes, so k_rescell3 sums each cell's contributions per corner, one wavefront per cell
// with a lane per (corner, point slot of 8) and a fixed butterfly over the slots, and
// k_resgather3 adds the 8 cell sums of every node.  Each record is read once instead of once per
// node it reaches (the node gather re-read 11 GB per launch on the 96^3 footing, half of it from
// HBM).  The cell sums [Ncell][8][4] (FP64) use the cell-matrix buffer, which the Jacobian only
// fills after the residual.
__global__ void __launch_bounds__(TPB) k_rescell3(Batch B) {
    const int q = batch_find(B, blockIdx.x);
    const Dev* __restrict__ d = B.d[q];
    const int64_t lb = blockIdx.x - B.pfx[q];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t c = lb * (TPB / 64) + wave;
    if (c >= d->Ncell) return;   // uniform over the wavefront
    using L = RecLayout<3, 2>;
    const int k = lane & 7, j = lane >> 3;   // corner (x + 2 y + 4 z), point slot
    const int kx = k & 1, ky = (k >> 1) & 1, kz = k >> 2;
    const int p0 = d->cstart[c], p1 = d->cstart[c + 1];
    const double pic = p1 > p0 ? d->cellpi[c * 8 + k] : 0.0;
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    for (int base = p0; base < p1; base += 8) {
        const int p = base + j;
        if (p >= p1) continue;
        const RecRef rc(d->rec, p, L::N);
        const double w[3] = {rc[L::W_ + kx], rc[L::W_ + 2 + ky], rc[L::W_ + 4 + kz]};
        const double dw[3] = {rc[L::DW_ + kx], rc[L::DW_ + 2 + ky], rc[L::DW_ + 4 + kz]};
        const double Sv = w[0] * w[1] * w[2];
        const double G[3] = {dw[0] * w[1] * w[2], w[0] * dw[1] * w[2], w[0] * w[1] * dw[2]};
        double gS[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double t = 0.0;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) t += rc[L::FI_ + cc * 3 + a] * G[cc];
            gS[a] = t;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double t = rc[L::BF_ + a] * Sv;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) t += rc[L::SG_ + a * 3 + cc] * gS[cc];
            r[a] += t;
        }
        double gw = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) gw += gS[a] * rc[L::QW_ + a];
        r[3] += Sv * rc[L::DT_] + rc[L::DK_] * gw + rc[L::ST_] * (Sv - pic);
    }
#pragma unroll
    for (int off = 8; off < 64; off <<= 1)
#pragma unroll
        for (int a = 0; a < 4; ++a) r[a] += __shfl_xor(r[a], off, 64);
    if (j == 0) {
        double* cr = (double*)d->Ke + (c * 8 + k) * 4;
#pragma unroll
        for (int a = 0; a < 4; ++a) cr[a] = r[a];
    }
}

__global__ void __launch_bounds__(TPB) k_resgather3(Batch B) {
    PROB_PROLOGUE
    double ru2 = 0.0, rp2 = 0.0;
    bool bad = false;
    if (tid < d->Nnode) {
        int n[3];
        n[0] = (int)(tid % d->nn[0]);
        n[1] = (int)((tid / d->nn[0]) % d->nn[1]);
        n[2] = (int)(tid / ((int64_t)d->nn[0] * d->nn[1]));
        const double* cr = (const double*)d->Ke;
        double r[4] = {0.0, 0.0, 0.0, 0.0};
        for (int kz = 0; kz < 2; ++kz)
            for (int ky = 0; ky < 2; ++ky)
                for (int kx = 0; kx < 2; ++kx) {
                    const int c0 = n[0] - kx, c1 = n[1] - ky, c2 = n[2] - kz;
                    if (c0 < 0 || c0 >= d->nc[0] || c1 < 0 || c1 >= d->nc[1] || c2 < 0 || c2 >= d->nc[2]) continue;
                    const int64_t c = c0 + (int64_t)d->nc[0] * (c1 + (int64_t)d->nc[1] * c2);
                    const double* v = cr + (c * 8 + kx + 2 * ky + 4 * kz) * 4;
#pragma unroll
                    for (int a = 0; a < 4; ++a) r[a] += v[a];
                }
        const int64_t pn = pad_index(d, n[0], n[1], n[2]);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            double v = r[a] + d->fext[pn * 4 + a];
            if (!d->dfree[pn * 4 + a]) v = 0.0;
            if (!isfinite(v)) bad = true;
            d->Rv[pn * 4 + a] = v;
            if (a < 3) ru2 += v * v;
            else rp2 += v * v;
        }
    }
    if (bad) atomicOr(&d->flags[FL_NONFINITE], 1);
    __shared__ double sh[2][TPB];
    sh[0][threadIdx.x] = ru2;
    sh[1][threadIdx.x] = rp2;
    __syncthreads();
    for (int off = TPB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + off];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        d->partial[lb * 4 + 0] = sh[0][0];
        d->partial[lb * 4 + 1] = sh[1][0];
    }
}

// Contribution of one point to the (ca, cc) entries of row node i, for every column node k of
// the point's window; LI is node i's window-local index (compile-time, so that the stencil slot
// of each k is a constant and the accumulators stay in registers).  With gi = dF^{-T} grad_n S_i,
// gk likewise, the (ca, cc) entry of J_ik is
//   ca, cc <  dim : gi . Abar_{ca . cc .} gk - d_ac m/(beta dt^2) S_i S_k
//   ca <  dim = cc: dv S_k gi_ca
//   ca = dim > cc : S_i (bv gk_cc - (LV^T gk)_cc) + dv kappa (gk_cc gi.w - gi_cc gk.w - gi.gk gp_cc)
//                   + dv kappa rho_f/(beta dt^2) gi_cc S_k  [+ dv J kappa'(J) gk_cc gi.w, Kozeny-Carman]
//   ca = cc = dim : dv kappa gi.gk + tau c_t V_n (S_i - Pi_i)(S_k - Pi_k)
// each written as u . gk + alpha S_k - gamma Pi_k = (f u) . grad_n S_k + alpha S_k - gamma Pi_k.
// pic: the cell's Pi S_k (original MPM, PPP class only).  C is the arithmetic type of the entries
// (double, or float for the FP32 Jacobian); the record fields are FP64 and are rounded on load.
template <int DIM, int SHAPE, int LI, typename C>
__device__ __forceinline__ void jac_point(const RecRef rc, const C* pic, int ca, int cc, bool kc,
                                          C* acc) {
    constexpr int WB = SHAPE ? 3 : 2;
    constexpr int RR = SHAPE ? 2 : 1;
    constexpr int SW = 2 * RR + 1;
    constexpr int NN = DIM == 2 ? WB * WB : WB * WB * WB;
    constexpr int li[3] = {LI % WB, (LI / WB) % WB, DIM == 3 ? LI / (WB * WB) : 0};
    using L = RecLayout<DIM, WB>;
    C w[DIM][WB], dw[DIM][WB];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int k = 0; k < WB; ++k) {
            w[a][k] = (C)rc[L::W_ + a * WB + k];
            dw[a][k] = (C)rc[L::DW_ + a * WB + k];
        }
    C Si = C(1), Gi[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) Si *= w[a][li[a]];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        C g = C(1);
#pragma unroll
        for (int c = 0; c < DIM; ++c) g *= (c == a) ? dw[c][li[c]] : w[c][li[c]];
        Gi[a] = g;
    }
    C f[DIM * DIM], gi[DIM];
#pragma unroll
    for (int e = 0; e < DIM * DIM; ++e) f[e] = (C)rc[L::FI_ + e];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        C t = C(0);
#pragma unroll
        for (int c = 0; c < DIM; ++c) t += f[c * DIM + a] * Gi[c];
        gi[a] = t;
    }
    C u[DIM], alpha = C(0), gamma = C(0), pik[NN];
#pragma unroll
    for (int k = 0; k < NN; ++k) pik[k] = C(0);
    const bool ppp = ca == DIM && cc == DIM;
    if (ca < DIM && cc < DIM) {
#pragma unroll
        for (int e = 0; e < DIM; ++e) {
            C t = C(0);
#pragma unroll
            for (int bb = 0; bb < DIM; ++bb) t += gi[bb] * (C)rc[L::AB_ + ((ca * DIM + bb) * DIM + cc) * DIM + e];
            u[e] = t;
        }
        if (ca == cc) alpha = -(C)rc[L::CM_] * Si;
    } else if (ca < DIM) {
#pragma unroll
        for (int e = 0; e < DIM; ++e) u[e] = C(0);
        C gia = C(0);
#pragma unroll
        for (int e = 0; e < DIM; ++e) gia += (e == ca) ? gi[e] : C(0);
        alpha = (C)rc[L::DV_] * gia;
    } else if (cc < DIM) {
        const C bv = (C)rc[L::BV_], dk = (C)rc[L::DK_];
        C qw[DIM], giq = C(0);
#pragma unroll
        for (int e = 0; e < DIM; ++e) {
            qw[e] = (C)rc[L::QW_ + e];
            giq += gi[e] * qw[e];
        }
        const C gpc = (C)rc[L::GP_ + cc];
        C gic = C(0);
#pragma unroll
        for (int e = 0; e < DIM; ++e) gic += (e == cc) ? gi[e] : C(0);
#pragma unroll
        for (int e = 0; e < DIM; ++e)
            u[e] = Si * ((e == cc ? bv : C(0)) - (C)rc[L::LV_ + e * DIM + cc]) +
                   dk * ((e == cc ? giq : C(0)) - gic * qw[e] - gi[e] * gpc);
        if (kc) u[cc] += (C)rc[L::KJ_] * giq;   // mobility varying with the volume ratio
        alpha = (C)rc[L::EE_] * gic;
    } else {
        const C dk = (C)rc[L::DK_];
#pragma unroll
        for (int e = 0; e < DIM; ++e) u[e] = dk * gi[e];
        if (SHAPE) {
            C s0[DIM][WB];
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int k = 0; k < WB; ++k) s0[a][k] = (C)rc[L::S0_ + a * WB + k];
#pragma unroll
            for (int k = 0; k < NN; ++k) {
                const int lk[3] = {k % WB, (k / WB) % WB, DIM == 3 ? k / (WB * WB) : 0};
                C v = C(1);
#pragma unroll
                for (int a = 0; a < DIM; ++a) v *= s0[a][lk[a]];
                pik[k] = v;
            }
        } else {
#pragma unroll
            for (int k = 0; k < NN; ++k) pik[k] = pic[k];
        }
        gamma = (C)rc[L::TC_] * (Si - pik[LI]);
        alpha = gamma;
    }
    C ut[DIM];
#pragma unroll
    for (int m = 0; m < DIM; ++m) {
        C t = C(0);
#pragma unroll
        for (int e = 0; e < DIM; ++e) t += f[m * DIM + e] * u[e];
        ut[m] = t;
    }
#pragma unroll
    for (int kz = 0; kz < (DIM == 3 ? WB : 1); ++kz)
#pragma unroll
        for (int ky = 0; ky < WB; ++ky)
#pragma unroll
            for (int kx = 0; kx < WB; ++kx) {
                const int s = (kx - li[0] + RR) + SW * (ky - li[1] + RR) +
                              (DIM == 3 ? SW * SW * (kz - li[2] + RR) : 0);
                const int kk = kx + WB * (ky + WB * kz);
                C val;
                if constexpr (DIM == 2) {
                    val = ut[0] * dw[0][kx] * w[1][ky] + ut[1] * w[0][kx] * dw[1][ky] + alpha * w[0][kx] * w[1][ky];
                } else {
                    val = ut[0] * dw[0][kx] * w[1][ky] * w[2][kz] + ut[1] * w[0][kx] * dw[1][ky] * w[2][kz] +
                          ut[2] * w[0][kx] * w[1][ky] * dw[2][kz] + alpha * w[0][kx] * w[1][ky] * w[2][kz];
                }
                if (ppp) val -= gamma * pik[kk];
                acc[s] += val;
            }
}

// All points of bucket n - l (LI = window index of n), then the next window index.
template <int DIM, int SHAPE, int LI, typename C>
__device__ __forceinline__ void jac_bucket(const Dev* __restrict__ d, const int* n, int ca, int cc, C* acc) {
    constexpr int WB = SHAPE ? 3 : 2;
    constexpr int NN = DIM == 2 ? WB * WB : WB * WB * WB;
    if constexpr (LI < NN) {
        using L = RecLayout<DIM, WB>;
        int64_t cid;
        int p0, p1;
        if (bucket_of<DIM, WB, LI>(d, n, &cid, &p0, &p1)) {
            C pic[NN];
#pragma unroll
            for (int k = 0; k < NN; ++k) pic[k] = C(0);
            if (!SHAPE && ca == DIM && cc == DIM && p1 > p0) {
#pragma unroll
                for (int k = 0; k < NN; ++k) pic[k] = (C)d->cellpi[cid * NN + k];
            }
            const bool kc = d->phi0 > C(0);
            for (int p = p0; p < p1; ++p) jac_point<DIM, SHAPE, LI, C>(RecRef(d->rec, p, L::N), pic, ca, cc, kc, acc);
        }
        jac_bucket<DIM, SHAPE, LI + 1, C>(d, n, ca, cc, acc);
    }
}

// Jacobian, one thread per (row node, ca, cc).  The b^2 component pairs of a node are adjacent
// lanes of one wavefront (64 / b^2 nodes per wavefront, consecutive in x), so that all lanes of a
// node read the same point record at the same time and a wavefront's record loads touch a few
// cache lines instead of one per lane.  The node's block row over the fixed stencil is
// accumulated in registers and written once, with the rows and columns of constrained dofs
// replaced by identity rows.  The point terms are formed and accumulated in T: the FP32 Jacobian
// of the mixed path (records, residual and Newton update stay FP64) needs about two thirds of
// the registers of the FP64 one and runs at 4-5 waves per SIMD instead of 3.
template <int DIM, int SHAPE, typename T>
__global__ void __launch_bounds__(TPB) k_jacobian(Batch B) {
    const int q = batch_find(B, blockIdx.x);
    const Dev* __restrict__ d = B.d[q];
    const int64_t lb = blockIdx.x - B.pfx[q];
    constexpr int RR = SHAPE ? 2 : 1;
    constexpr int SW = 2 * RR + 1;
    constexpr int S = DIM == 2 ? SW * SW : SW * SW * SW;
    constexpr int BS = DIM + 1;
    constexpr int NP = BS * BS;
    constexpr int NPW = 64 / NP;                 // nodes per wavefront
    constexpr int NODES = (TPB / 64) * NPW;      // nodes per block (an x-run)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane >= NP * NPW) return;
    const int pair = lane % NP;
    const int ca = pair / BS, cc = pair % BS;
    const int ntx = (d->nn[0] + NODES - 1) / NODES;
    int n[3];
    n[0] = (int)(lb % ntx) * NODES + wave * NPW + lane / NP;
    n[1] = (int)((lb / ntx) % d->nn[1]);
    n[2] = DIM == 3 ? (int)(lb / ((int64_t)ntx * d->nn[1])) : 0;
    if (n[0] >= d->nn[0]) return;
    const int64_t row = n[0] + (int64_t)d->nn[0] * (n[1] + (int64_t)d->nn[1] * n[2]);
    T acc[S];   // accumulated, like the point terms, in the Jacobian's own precision
#pragma unroll
    for (int s = 0; s < S; ++s) acc[s] = T(0);
    jac_bucket<DIM, SHAPE, 0, T>(d, n, ca, cc, acc);
    const int64_t pni = pad_index(d, n[0], n[1], n[2]);
    const bool fr = d->dfree[pni * BS + ca] != 0;
    T* J = (T*)d->J;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const int off[3] = {s % SW - RR, (s / SW) % SW - RR, DIM == 3 ? s / (SW * SW) - RR : 0};
        bool valid = true;
        int k[3] = {0, 0, 0};
        for (int a = 0; a < DIM; ++a) {
            k[a] = n[a] + off[a];
            if (k[a] < 0 || k[a] >= d->nn[a]) valid = false;
        }
        double v = 0.0;
        if (valid) {
            v = acc[s];
            const int64_t pnk = pad_index(d, k[0], k[1], k[2]);
            const bool fc = d->dfree[pnk * BS + cc] != 0;
            if (!(fr && fc)) v = (s == (S - 1) / 2 && ca == cc) ? 1.0 : 0.0;
        }
        J[jidx<DIM>((s * BS + ca) * BS + cc, row, S * BS * BS, d->Nnode)] = (T)v;
    }
}

// ---------------------------------------------------------------------------------------------
// 3D Jacobian: cell matrices, then block rows
// ---------------------------------------------------------------------------------------------
// Trilinear basis: the points of cell c (its sort bucket) reach exactly the cell's 8 corner
// nodes, so the Jacobian is the sum of cell matrices K_c = sum_{p in c} (point terms), each
// 8 x 8 blocks of 4 x 4.  k_cellmat3 forms them with one wavefront per cell and one lane per
// node pair (i, k) of the cell (lane = 8 i + k, corner index x + 2 y + 4 z): the cell's points
// are walked in order at wave-uniform addresses, so every lane reads the same record words and
// computes its own 16 entries from them (no atomics, no redundant point terms); the lanes store
// K_c as Ke[(c * 16 + e) * 64 + lane], 64 consecutive words per entry.  With gi = dF^{-T} grad_n S_i
// (likewise gk), the (a, c) entries of the block J_ik are
//   uu  -V0 G (gi . b gk) d_ac + C1 gk_a gi_c + C2 gi_a gk_c - m/(beta dt^2) S_i S_k d_ac
//       [Kelvin damping, with l the velocity gradient and v_g = gamma/(beta dt):
//        - alpha (lam gi_a (dv v_g gk_c - (dv l^T gk)_c) + G (gi . gk)(dv v_g d_ac - dv l_ac)
//                 + G gk_a (dv v_g gi_c - (dv l^T gi)_c)) - dv (s_vis gi)_a gk_c + dv (s_vis gk)_a gi_c]
//   up  dv S_k gi_a
//   pu  S_i (bv gk_c - (dv l^T gk)_c) + dv kappa (gk_c gi.w - gi_c w.gk - (gi . gk) gp_c)
//       + dv kappa rho_f/(beta dt^2) gi_c S_k  [+ dv J kappa'(J) (gi.w) gk_c, Kozeny-Carman]
//   pp  dv kappa gi . gk + tau c_t V_n (S_i - Pi_i)(S_k - Pi_k)
// (the exact derivatives of the residual terms listed at the top of this file; the same
// entries as the 2D kernel's folded-tangent form).  T is the Jacobian's precision.
template <typename T, bool DYN, bool VIS>
__global__ void __launch_bounds__(TPB) k_cellmat3(Batch B) {
    const int q = batch_find(B, blockIdx.x);
    const Dev* __restrict__ d = B.d[q];
    const int64_t lb = blockIdx.x - B.pfx[q];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t c = lb * (TPB / 64) + wave;
    if (c >= d->Ncell) return;
    // wave-uniform point range (readfirstlane: the compiler then keeps the record addresses scalar)
    const int p0 = __builtin_amdgcn_readfirstlane(d->cstart[c]);
    const int p1 = __builtin_amdgcn_readfirstlane(d->cstart[c + 1]);
    using L = RecLayout<3, 2>;   // (an empty cell stores a zero matrix)
    const int i = lane >> 3, k = lane & 7;
    const int ix = i & 1, iy = (i >> 1) & 1, iz = i >> 2;
    const int kx = k & 1, ky = (k >> 1) & 1, kz = k >> 2;
    const T Pii = (T)d->cellpi[c * 8 + i], Pik = (T)d->cellpi[c * 8 + k];
    const bool kc = d->phi0 > 0.0;
    const T lam = (T)d->lam, Gm = (T)d->G, al = (T)d->alpha_vis, vg = (T)(d->gamma / (d->beta * d->dt));
    T acc[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[e] = T(0);
    // the records are read-only here and every lane reads the same words: the constant address
    // space turns them into scalar loads (written by the records kernel, a previous launch)
    using CRec = const __attribute__((address_space(4))) double*;
    const CRec rec = (CRec)d->rec;
    for (int p = p0; p < p1; ++p) {
        const CRec r = rec + (int64_t)p * L::N;
        // basis of nodes i and k (reference gradients), then spatial gradients gi, gk; the 1D
        // values are loaded for both nodes of each axis (uniform) and selected per lane
        T w1[6], d1[6];
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            w1[e] = (T)r[L::W_ + e];
            d1[e] = (T)r[L::DW_ + e];
        }
        const T wxi = ix ? w1[1] : w1[0], wyi = iy ? w1[3] : w1[2], wzi = iz ? w1[5] : w1[4];
        const T dxi = ix ? d1[1] : d1[0], dyi = iy ? d1[3] : d1[2], dzi = iz ? d1[5] : d1[4];
        const T wxk = kx ? w1[1] : w1[0], wyk = ky ? w1[3] : w1[2], wzk = kz ? w1[5] : w1[4];
        const T dxk = kx ? d1[1] : d1[0], dyk = ky ? d1[3] : d1[2], dzk = kz ? d1[5] : d1[4];
        const T Si = wxi * wyi * wzi, Sk = wxk * wyk * wzk;
        const T Gi[3] = {dxi * wyi * wzi, wxi * dyi * wzi, wxi * wyi * dzi};
        const T Gk[3] = {dxk * wyk * wzk, wxk * dyk * wzk, wxk * wyk * dzk};
        T f[9];
#pragma unroll
        for (int e = 0; e < 9; ++e) f[e] = (T)r[L::FI_ + e];
        T gi[3], gk[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            gi[a] = f[a] * Gi[0] + f[3 + a] * Gi[1] + f[6 + a] * Gi[2];
            gk[a] = f[a] * Gk[0] + f[3 + a] * Gk[1] + f[6 + a] * Gk[2];
        }
        const T dv = (T)r[L::DV_];
        const T b00 = (T)r[L::BM_ + 0], b11 = (T)r[L::BM_ + 1], b22 = (T)r[L::BM_ + 2];
        const T b01 = (T)r[L::BM_ + 3], b12 = (T)r[L::BM_ + 4], b02 = (T)r[L::BM_ + 5];
        const T bgk[3] = {b00 * gk[0] + b01 * gk[1] + b02 * gk[2], b01 * gk[0] + b11 * gk[1] + b12 * gk[2],
                          b02 * gk[0] + b12 * gk[1] + b22 * gk[2]};
        const T gbg = gi[0] * bgk[0] + gi[1] * bgk[1] + gi[2] * bgk[2];
        const T gigk = gi[0] * gk[0] + gi[1] * gk[1] + gi[2] * gk[2];
        T diag = -(T)r[L::VG_] * gbg;
        if (DYN) diag -= (T)r[L::CM_] * Si * Sk;
        const T C1 = (T)r[L::C1_], C2 = (T)r[L::C2_];
        T LV[9], lti[3], ltk[3];
        if (DYN) {
#pragma unroll
            for (int e = 0; e < 9; ++e) LV[e] = (T)r[L::LV_ + e];
#pragma unroll
            for (int a = 0; a < 3; ++a) {   // (dv l^T g)_a = sum_e LV[e][a] g_e
                ltk[a] = LV[a] * gk[0] + LV[3 + a] * gk[1] + LV[6 + a] * gk[2];
                lti[a] = LV[a] * gi[0] + LV[3 + a] * gi[1] + LV[6 + a] * gi[2];
            }
        }
        // displacement-displacement block
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                T v = C1 * gk[a] * gi[cc] + C2 * gi[a] * gk[cc];
                if (a == cc) v += diag;
                acc[a * 4 + cc] += v;
            }
        if (VIS) {
            const T s00 = (T)r[L::SV_ + 0], s11 = (T)r[L::SV_ + 1], s22 = (T)r[L::SV_ + 2];
            const T s01 = (T)r[L::SV_ + 3], s12 = (T)r[L::SV_ + 4], s02 = (T)r[L::SV_ + 5];
            const T sgi[3] = {s00 * gi[0] + s01 * gi[1] + s02 * gi[2], s01 * gi[0] + s11 * gi[1] + s12 * gi[2],
                              s02 * gi[0] + s12 * gi[1] + s22 * gi[2]};
            const T sgk[3] = {s00 * gk[0] + s01 * gk[1] + s02 * gk[2], s01 * gk[0] + s11 * gk[1] + s12 * gk[2],
                              s02 * gk[0] + s12 * gk[1] + s22 * gk[2]};
            const T dvg = dv * vg;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    T t = lam * gi[a] * (dvg * gk[cc] - ltk[cc]) + Gm * gigk * ((a == cc ? dvg : T(0)) - LV[a * 3 + cc]) +
                          Gm * gk[a] * (dvg * gi[cc] - lti[cc]);
                    acc[a * 4 + cc] += -al * t - dv * sgi[a] * gk[cc] + dv * sgk[a] * gi[cc];
                }
        }
        // displacement rows, pressure column
        const T dvs = dv * Sk;
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[a * 4 + 3] += dvs * gi[a];
        // pressure row, displacement columns
        const T bv = (T)r[L::BV_], dk = (T)r[L::DK_];
        const T qw[3] = {(T)r[L::QW_], (T)r[L::QW_ + 1], (T)r[L::QW_ + 2]};
        const T giq = gi[0] * qw[0] + gi[1] * qw[1] + gi[2] * qw[2];
        const T qwk = qw[0] * gk[0] + qw[1] * gk[1] + qw[2] * gk[2];
        T gkc = Si * bv + dk * giq;
        if (kc) gkc += (T)r[L::KJ_] * giq;
        const T gic = -dk * qwk + (DYN ? (T)r[L::EE_] * Sk : T(0));
        const T gpf = -dk * gigk;
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            T v = gkc * gk[cc] + gic * gi[cc] + gpf * (T)r[L::GP_ + cc];
            if (DYN) v -= Si * ltk[cc];
            acc[12 + cc] += v;
        }
        // pressure-pressure
        acc[15] += dk * gigk + (T)r[L::TC_] * (Si - Pii) * (Sk - Pik);
    }
    using GT = __attribute__((address_space(1))) T*;
    const GT Ke = (GT)d->Ke;
#pragma unroll
    for (int e = 0; e < 16; ++e) Ke[(c * 16 + e) * 64 + lane] = acc[e];
}

// Block rows of the 3D Jacobian from the cell matrices: a wavefront per (run of 64 consecutive
// nodes along x, block entry e = 4 a + c), a thread per node.  The node is corner i of its cells
// c = n - i; their blocks (i, k) go to the stencil slots k - i, summed over i in a fixed order.
// Rows and columns of constrained dofs become identity rows; each store writes 64 consecutive
// rows of one entry.
template <typename T>
__global__ void __launch_bounds__(TPB) k_jacgather3(Batch B) {
    const int q = batch_find(B, blockIdx.x);
    const Dev* __restrict__ d = B.d[q];
    const int64_t lb = blockIdx.x - B.pfx[q];
    const int64_t W = lb * (TPB / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int e = (int)(W % 16), ca = e >> 2, cc = e & 3;
    const int64_t run = W / 16;
    const int nrx = (d->nn[0] + 63) / 64;
    const int x = (int)(run % nrx) * 64 + lane;
    const int y = (int)((run / nrx) % d->nn[1]);
    const int z = (int)(run / ((int64_t)nrx * d->nn[1]));
    if (z >= d->nn[2] || x >= d->nn[0]) return;
    using GT = const __attribute__((address_space(1))) T*;
    const GT Ke = (GT)d->Ke;
    T acc[27];
#pragma unroll
    for (int s = 0; s < 27; ++s) acc[s] = T(0);
    // branch-free over the 8 cells (an off-grid cell reads cell 0 with weight 0), so that all
    // loads issue together; node n's entries (i, 0..7) of a cell and its x-neighbour's (i ^ 1,
    // 0..7) share a 128-byte line
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int ix = i & 1, iy = (i >> 1) & 1, iz = i >> 2;
        const int cx = x - ix, cy = y - iy, cz = z - iz;
        const bool in = cx >= 0 && cy >= 0 && cz >= 0 && cx < d->nc[0] && cy < d->nc[1] && cz < d->nc[2];
        const int64_t c = in ? cx + (int64_t)d->nc[0] * (cy + (int64_t)d->nc[1] * cz) : 0;
        const T wgt = in ? T(1) : T(0);
        const GT kp = Ke + (c * 16 + e) * 64 + i * 8;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int kx = k & 1, ky = (k >> 1) & 1, kz = k >> 2;
            acc[(kx - ix + 1) + 3 * ((ky - iy + 1) + 3 * (kz - iz + 1))] += wgt * kp[k];
        }
    }
    const int64_t row = x + (int64_t)d->nn[0] * (y + (int64_t)d->nn[1] * z);
    const int64_t pni = pad_index(d, x, y, z);
    const bool fr = d->dfree[pni * 4 + ca] != 0;
    T* __restrict__ J = (T*)d->J;
#pragma unroll
    for (int s = 0; s < 27; ++s) {
        const int ox = s % 3 - 1, oy = (s / 3) % 3 - 1, oz = s / 9 - 1;
        const int kx = x + ox, ky = y + oy, kz = z + oz;
        const bool valid = kx >= 0 && ky >= 0 && kz >= 0 && kx < d->nn[0] && ky < d->nn[1] && kz < d->nn[2];
        T v = T(0);
        if (valid) {
            v = acc[s];
            const bool fc = d->dfree[pad_index(d, kx, ky, kz) * 4 + cc] != 0;
            if (!(fr && fc)) v = (s == 13 && ca == cc) ? T(1) : T(0);
        }
        J[jidx<3>((s * 4 + ca) * 4 + cc, row, 27 * 16, d->Nnode)] = v;
    }
}

// sum of the residual partials of each problem (one block per problem)
__global__ void k_finalize_norms(Batch B) {
    const int q = blockIdx.x;
    const Dev* d = B.d[q];
    __shared__ double sh[2][TPB];
    double a = 0.0, b2 = 0.0;
    const int64_t nblk = B.pfx[q + 1] - B.pfx[q];   // blocks of k_residual for this problem
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
    if (threadIdx.x == 0) {
        d->scal[SC_RU2] = sh[0][0];
        d->scal[SC_RP2] = sh[1][0];
    }
}

// ---------------------------------------------------------------------------------------------
void launch_assemble(const Group& g, bool want_J, hipStream_t st) {
    Batch Bp = make_batch(g.ddev, g.np, TPB);
    Batch Bn = make_batch_blocks(g.ddev, g.ntile);
    if (g.dim == 2 && g.shape == 0) {
        PPM_TIMED(KT_RECORDS, st, hipLaunchKernelGGL((k_records<2, 0>), dim3(Bp.pfx[Bp.n]), dim3(TPB), 0, st, Bp));
        PPM_TIMED(KT_RESIDUAL, st, hipLaunchKernelGGL((k_residual<2, 0>), dim3(Bn.pfx[Bn.n]), dim3(TPB), 0, st, Bn));
    } else if (g.dim == 2 && g.shape == 1) {
        PPM_TIMED(KT_RECORDS, st, hipLaunchKernelGGL((k_records<2, 1>), dim3(Bp.pfx[Bp.n]), dim3(TPB), 0, st, Bp));
        PPM_TIMED(KT_RESIDUAL, st, hipLaunchKernelGGL((k_residual<2, 1>), dim3(Bn.pfx[Bn.n]), dim3(TPB), 0, st, Bn));
    } else {
        PPM_TIMED(KT_RECORDS, st, hipLaunchKernelGGL((k_records<3, 0>), dim3(Bp.pfx[Bp.n]), dim3(TPB), 0, st, Bp));
        std::vector<int64_t> cw;
        for (size_t q = 0; q < g.ddev.size(); ++q) cw.push_back((g.ncell[q] + TPB / 64 - 1) / (TPB / 64));
        Batch Bc = make_batch_blocks(g.ddev, cw);
        Batch Bg = make_batch(g.ddev, g.nnode, TPB);
        PPM_TIMED(KT_RESIDUAL, st, hipLaunchKernelGGL(k_rescell3, dim3(Bc.pfx[Bc.n]), dim3(TPB), 0, st, Bc);
                  hipLaunchKernelGGL(k_resgather3, dim3(Bg.pfx[Bg.n]), dim3(TPB), 0, st, Bg));
        hipLaunchKernelGGL(k_finalize_norms, dim3(Bg.n), dim3(TPB), 0, st, Bg);
        if (want_J) launch_jacobian(g, st);
        return;
    }
    hipLaunchKernelGGL(k_finalize_norms, dim3(Bn.n), dim3(TPB), 0, st, Bn);
    if (want_J) launch_jacobian(g, st);
}

void launch_jacobian(const Group& g, hipStream_t st) {
    Batch Bn = make_batch_blocks(g.ddev, g.jblk);
    const dim3 gr(Bn.pfx[Bn.n]), tb(TPB);
    if (g.dim == 2 && g.shape == 0) {
        if (g.mixed) PPM_TIMED(KT_JACOBIAN, st, hipLaunchKernelGGL((k_jacobian<2, 0, float>), gr, tb, 0, st, Bn));
        else PPM_TIMED(KT_JACOBIAN, st, hipLaunchKernelGGL((k_jacobian<2, 0, double>), gr, tb, 0, st, Bn));
    } else if (g.dim == 2 && g.shape == 1) {
        if (g.mixed) PPM_TIMED(KT_JACOBIAN, st, hipLaunchKernelGGL((k_jacobian<2, 1, float>), gr, tb, 0, st, Bn));
        else PPM_TIMED(KT_JACOBIAN, st, hipLaunchKernelGGL((k_jacobian<2, 1, double>), gr, tb, 0, st, Bn));
    } else {
        // cell matrices (a wavefront per cell), then the block rows (a wavefront per 64-node run
        // and block entry)
        std::vector<int64_t> cw, gw;
        bool dyn = false, vis = false;
        for (size_t i = 0; i < g.ncell.size(); ++i) {
            cw.push_back(g.ncell[i] * 64);
            gw.push_back(jacgather3_blocks(g.nn3[i]));
        }
        for (const Dev* hd : g.hdev) {
            dyn = dyn || hd->dyn;
            vis = vis || (hd->dyn && hd->alpha_vis != 0.0);
        }
        Batch Bc = make_batch(g.ddev, cw, TPB);
        Batch Bg = make_batch_blocks(g.ddev, gw);
        const dim3 gc(Bc.pfx[Bc.n]), gg(Bg.pfx[Bg.n]);
        if (g.mixed) {
            if (vis) PPM_TIMED(KT_CELLMAT, st, hipLaunchKernelGGL((k_cellmat3<float, true, true>), gc, tb, 0, st, Bc));
            else if (dyn) PPM_TIMED(KT_CELLMAT, st, hipLaunchKernelGGL((k_cellmat3<float, true, false>), gc, tb, 0, st, Bc));
            else PPM_TIMED(KT_CELLMAT, st, hipLaunchKernelGGL((k_cellmat3<float, false, false>), gc, tb, 0, st, Bc));
            PPM_TIMED(KT_JACOBIAN, st, hipLaunchKernelGGL((k_jacgather3<float>), gg, tb, 0, st, Bg));
        } else {
            if (vis) PPM_TIMED(KT_CELLMAT, st, hipLaunchKernelGGL((k_cellmat3<double, true, true>), gc, tb, 0, st, Bc));
            else if (dyn) PPM_TIMED(KT_CELLMAT, st, hipLaunchKernelGGL((k_cellmat3<double, true, false>), gc, tb, 0, st, Bc));
            else PPM_TIMED(KT_CELLMAT, st, hipLaunchKernelGGL((k_cellmat3<double, false, false>), gc, tb, 0, st, Bc));
            PPM_TIMED(KT_JACOBIAN, st, hipLaunchKernelGGL((k_jacgather3<double>), gg, tb, 0, st, Bg));
        }
    }
}

}  // namespace ppm
