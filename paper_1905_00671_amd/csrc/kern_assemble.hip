// Residual and Jacobian assembly at the material points (Sec. 3.1-3.4, Sec. 4.2).
//
// Two passes per Newton iteration:
//   k_records   one thread per (sorted) material point: basis at x_n, relative deformation
//               dF = 1 + sum U (x) grad_n S, stress, tangent and every per-point coefficient the
//               residual and the Jacobian need ("quadrature record", SoA in HBM);
//   k_residual  one thread per grid node: gathers R_i from the points whose basis reaches node i
//               (no atomics, fixed summation order), applies the boundary conditions and writes
//               per-block partial norms;
//   k_jacobian  one thread per (grid node i, stencil neighbour k): gathers the 3x3 / 4x4 block
//               J_ik from the points shared by both nodes and writes it once into the
//               fixed-stencil block rows (no atomics).
// Residual terms (current configuration, dv = det(dF) V_n, grad S = dF^{-T} grad_n S):
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

template <int DIM, int SHAPE>
__global__ void __launch_bounds__(TPB) k_records(Batch B) {
    PROB_PROLOGUE
    if (tid >= d->Np) return;
    constexpr int WB = SHAPE ? 3 : 2;
    constexpr int NN = DIM == 2 ? WB * WB : WB * WB * WB;
    using L = RecLayout<DIM, WB>;
    const int bs = DIM + 1;
    const double* P = d->pw;
    const int64_t s = d->ps, Np = d->Np;
    const int64_t i = tid;
    double* rec = d->rec;
    double w[DIM][3], dw[DIM][3], s0v[DIM][3];
    int base[3] = {0, 0, 0};
    for (int a = 0; a < DIM; ++a) {
        base[a] = basis_1d<SHAPE>(P[(PX + a) * s + i], P[(PLP + a) * s + i], d->x0[a], d->h, d->nc[a], w[a],
                                  dw[a], s0v[a]);
        d->rbase[a * Np + i] = base[a];
        for (int k = 0; k < WB; ++k) {
            rec[(L::W_ + a * WB + k) * Np + i] = w[a][k];
            rec[(L::DW_ + a * WB + k) * Np + i] = dw[a][k];
            rec[(L::S0_ + a * WB + k) * Np + i] = s0v[a][k];
        }
    }
    int64_t cid = 0;
    if (SHAPE == 0) {
        int64_t mul = 1;
        for (int a = 0; a < DIM; ++a) { cid += base[a] * mul; mul *= d->nc[a]; }
    }
    const double dt = d->dt, be = d->beta, ga = d->gamma;
    const bool dyn = d->dyn;
    double G[NN][DIM], Sv[NN], Pi[NN], U[NN][DIM], Pk[NN], acc[NN][DIM], vel[NN][DIM], pdot[NN];
    double dF[DIM * DIM];
    for (int k = 0; k < DIM * DIM; ++k) dF[k] = (k % (DIM + 1) == 0) ? 1.0 : 0.0;
    for (int k = 0; k < NN; ++k) {
        int li[3] = {k % WB, (k / WB) % WB, DIM == 3 ? k / (WB * WB) : 0};
        double sv = 1.0, s0p = 1.0;
        for (int a = 0; a < DIM; ++a) {
            sv *= w[a][li[a]];
            s0p *= s0v[a][li[a]];
            double gr = 1.0;
            for (int c = 0; c < DIM; ++c) gr *= (c == a) ? dw[c][li[c]] : w[c][li[c]];
            G[k][a] = gr;
        }
        Sv[k] = sv;
        Pi[k] = SHAPE ? s0p : d->cellpi[cid * (1 << DIM) + k];
        int64_t pn = pad_index(d, base[0] + li[0], base[1] + li[1], DIM == 3 ? base[2] + li[2] : 0);
        const double* Xn = d->X + pn * bs;
        for (int a = 0; a < DIM; ++a) U[k][a] = Xn[a];
        Pk[k] = Xn[DIM];
        for (int a = 0; a < DIM; ++a)
            for (int c = 0; c < DIM; ++c) dF[a * DIM + c] += U[k][a] * G[k][c];
        double dP = Pk[k] - d->Pn[pn];
        pdot[k] = d->ct * dP;
        if (dyn) {
            pdot[k] += d->hc1 * d->pdn[pn] + d->hc2 * d->pddn[pn];
            for (int a = 0; a < DIM; ++a) {
                double v0 = d->vn[pn * 3 + a], a0 = d->an[pn * 3 + a];
                acc[k][a] = U[k][a] / (be * dt * dt) - v0 / (be * dt) + (1.0 - 0.5 / be) * a0;
                vel[k][a] = ga / (be * dt) * U[k][a] + (1.0 - ga / be) * v0 + (1.0 - 0.5 * ga / be) * dt * a0;
            }
        }
    }
    double dJ = det<DIM>(dF);
    if (!(dJ > 0.0)) {
        atomicOr(&d->flags[FL_INVERTED], 1);
        dJ = 1.0;
        for (int k = 0; k < DIM * DIM; ++k) dF[k] = (k % (DIM + 1) == 0) ? 1.0 : 0.0;
    }
    double f[DIM * DIM], Fn[DIM * DIM], F[DIM * DIM];
    inverse<DIM>(dF, f);
    for (int k = 0; k < DIM * DIM; ++k) Fn[k] = P[(PF + k) * s + i];
    for (int a = 0; a < DIM; ++a)
        for (int c = 0; c < DIM; ++c) {
            double t = 0.0;
            for (int k = 0; k < DIM; ++k) t += dF[a * DIM + k] * Fn[k * DIM + c];
            F[a * DIM + c] = t;
        }
    double tau[DIM * DIM], tzz, T[DIM * DIM * DIM * DIM];
    kirchhoff_tangent<DIM>(d->model, d->lam, d->G, F, tau, &tzz, T);
    const double Vn = P[PV * s + i], m = P[PM * s + i];
    const double V0 = Vn / det<DIM>(Fn);
    const double dv = dJ * Vn;
    double gS[NN][DIM];
    double ph = 0.0, gp[DIM], ah[DIM], l[DIM * DIM];
    for (int a = 0; a < DIM; ++a) gp[a] = ah[a] = 0.0;
    for (int k = 0; k < DIM * DIM; ++k) l[k] = 0.0;
    double pst = 0.0;
    for (int k = 0; k < NN; ++k) {
        for (int a = 0; a < DIM; ++a) {
            double t = 0.0;
            for (int c = 0; c < DIM; ++c) t += f[c * DIM + a] * G[k][c];
            gS[k][a] = t;
        }
        ph += Sv[k] * Pk[k];
        for (int a = 0; a < DIM; ++a) gp[a] += Pk[k] * gS[k][a];
        pst += (Sv[k] - Pi[k]) * pdot[k];
        if (dyn) {
            for (int a = 0; a < DIM; ++a) {
                ah[a] += Sv[k] * acc[k][a];
                for (int c = 0; c < DIM; ++c) l[a * DIM + c] += vel[k][a] * gS[k][c];
            }
        }
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
    // tangent with the geometric term and the pressure term folded in
    for (int a = 0; a < DIM; ++a)
        for (int bb = 0; bb < DIM; ++bb)
            for (int c = 0; c < DIM; ++c)
                for (int e = 0; e < DIM; ++e) {
                    double v = -V0 * T[((a * DIM + bb) * DIM + c) * DIM + e];
                    if (bb == c) v += V0 * tau[a * DIM + e];
                    if (a == bb && c == e) v += dv * ph;
                    if (a == e && bb == c) v -= dv * ph;
                    rec[(L::AB_ + ((a * DIM + bb) * DIM + c) * DIM + e) * Np + i] = v;
                }
    for (int k = 0; k < DIM * DIM; ++k) {
        rec[(L::FI_ + k) * Np + i] = f[k];
        rec[(L::LV_ + k) * Np + i] = dyn ? dv * l[k] : 0.0;
        int a = k / DIM, c = k % DIM;
        rec[(L::SG_ + k) * Np + i] = -V0 * tau[k] + (a == c ? dv * ph : 0.0);
    }
    rec[L::DV_ * Np + i] = dv;
    rec[L::CM_ * Np + i] = dyn ? m / (be * dt * dt) : 0.0;
    rec[L::BV_ * Np + i] = dyn ? dv * (theta + ga / (be * dt)) : dv * (1.0 + log(dJ)) / dt;
    rec[L::DK_ * Np + i] = dv * d->kappa;
    for (int a = 0; a < DIM; ++a) {
        rec[(L::GP_ + a) * Np + i] = gp[a];
        rec[(L::QW_ + a) * Np + i] = wv[a];
        rec[(L::BF_ + a) * Np + i] = m * (d->g[a] - ah[a]);
    }
    rec[L::EE_ * Np + i] = dyn ? dv * d->kappa * d->rho_f / (be * dt * dt) : 0.0;
    rec[L::TC_ * Np + i] = d->tau * d->ct * Vn;
    rec[L::DT_ * Np + i] = dv * theta;
    rec[L::ST_ * Np + i] = d->tau * Vn * pst;
}

// S, grad_n S of node (li) from a record, for a point with window-local node index li[]
template <int DIM, int WB>
__device__ __forceinline__ void rec_basis(const double* __restrict__ rec, int64_t Np, int64_t p,
                                          const int* li, double& Sv, double* G, double& s0) {
    using L = RecLayout<DIM, WB>;
    double w[DIM], dw[DIM];
    Sv = 1.0;
    s0 = 1.0;
    for (int a = 0; a < DIM; ++a) {
        w[a] = rec[(L::W_ + a * WB + li[a]) * Np + p];
        dw[a] = rec[(L::DW_ + a * WB + li[a]) * Np + p];
        s0 *= rec[(L::S0_ + a * WB + li[a]) * Np + p];
        Sv *= w[a];
    }
    for (int a = 0; a < DIM; ++a) {
        double g = 1.0;
        for (int c = 0; c < DIM; ++c) g *= (c == a) ? dw[c] : w[c];
        G[a] = g;
    }
}

template <int DIM>
__device__ __forceinline__ void node_coords(const Dev* d, int64_t row, int* n) {
    n[0] = (int)(row % d->nn[0]);
    n[1] = (int)((row / d->nn[0]) % d->nn[1]);
    n[2] = DIM == 3 ? (int)(row / ((int64_t)d->nn[0] * d->nn[1])) : 0;
}

template <int DIM, int SHAPE>
__global__ void __launch_bounds__(TPB) k_residual(Batch B) {
    PROB_PROLOGUE
    constexpr int WB = SHAPE ? 3 : 2;
    using L = RecLayout<DIM, WB>;
    const int bs = DIM + 1;
    double ru2 = 0.0, rp2 = 0.0;
    bool bad = false;
    if (tid < d->Nnode) {
        int n[3];
        node_coords<DIM>(d, tid, n);
        const int64_t pn = pad_index(d, n[0], n[1], n[2]);
        const double* __restrict__ rec = d->rec;
        const int64_t Np = d->Np;
        int clo[3] = {0, 0, 0}, chi[3] = {0, 0, 0};
        for (int a = 0; a < DIM; ++a) {
            clo[a] = max(n[a] - (SHAPE ? 2 : 1), 0);
            chi[a] = min(n[a] + (SHAPE ? 1 : 0), d->nc[a] - 1);
        }
        double r[DIM + 1];
        for (int c = 0; c <= DIM; ++c) r[c] = 0.0;
        for (int cz = (DIM == 3 ? clo[2] : 0); cz <= (DIM == 3 ? chi[2] : 0); ++cz)
            for (int cy = clo[1]; cy <= chi[1]; ++cy) {
                int64_t rowc = (int64_t)d->nc[0] * (cy + (int64_t)d->nc[1] * cz);
                int p0 = d->cstart[rowc + clo[0]], p1 = d->cstart[rowc + chi[0] + 1];
                for (int p = p0; p < p1; ++p) {
                    int li[3] = {0, 0, 0};
                    bool in = true;
                    for (int a = 0; a < DIM; ++a) {
                        li[a] = n[a] - d->rbase[a * Np + p];
                        if (li[a] < 0 || li[a] >= WB) in = false;
                    }
                    if (!in) continue;
                    double Sv, G[DIM], s0;
                    rec_basis<DIM, WB>(rec, Np, p, li, Sv, G, s0);
                    double gS[DIM];
                    for (int a = 0; a < DIM; ++a) {
                        double t = 0.0;
                        for (int c = 0; c < DIM; ++c) t += rec[(L::FI_ + c * DIM + a) * Np + p] * G[c];
                        gS[a] = t;
                    }
                    for (int a = 0; a < DIM; ++a) {
                        double t = rec[(L::BF_ + a) * Np + p] * Sv;
                        for (int c = 0; c < DIM; ++c) t += rec[(L::SG_ + a * DIM + c) * Np + p] * gS[c];
                        r[a] += t;
                    }
                    double Pi;
                    if (SHAPE) {
                        Pi = s0;
                    } else {
                        int64_t cid = 0, mul = 1, lin = 0;
                        for (int a = 0; a < DIM; ++a) {
                            cid += d->rbase[a * Np + p] * mul;
                            mul *= d->nc[a];
                            lin += (int64_t)li[a] << a;
                        }
                        Pi = d->cellpi[cid * (1 << DIM) + lin];
                    }
                    double gw = 0.0;
                    for (int a = 0; a < DIM; ++a) gw += gS[a] * rec[(L::QW_ + a) * Np + p];
                    r[DIM] += Sv * rec[L::DT_ * Np + p] + rec[L::DK_ * Np + p] * gw + rec[L::ST_ * Np + p] * (Sv - Pi);
                }
            }
        for (int c = 0; c <= DIM; ++c) {
            double v = r[c] + d->fext[pn * bs + c];
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

// Jacobian block J_ik for row node i and stencil neighbour k = i + offset(blockIdx.y).
template <int DIM, int SHAPE, typename T>
__global__ void __launch_bounds__(TPB) k_jacobian(Batch B) {
    PROB_PROLOGUE
    if (tid >= d->Nnode) return;
    constexpr int WB = SHAPE ? 3 : 2;
    constexpr int RR = SHAPE ? 2 : 1;
    constexpr int SW = 2 * RR + 1;
    constexpr int BS = DIM + 1;
    using L = RecLayout<DIM, WB>;
    const int sidx = blockIdx.y;
    int off[3] = {sidx % SW - RR, (sidx / SW) % SW - RR, DIM == 3 ? sidx / (SW * SW) - RR : 0};
    int n[3], k[3];
    node_coords<DIM>(d, tid, n);
    bool valid = true;
    for (int a = 0; a < DIM; ++a) {
        k[a] = n[a] + off[a];
        if (k[a] < 0 || k[a] >= d->nn[a]) valid = false;
    }
    double blk[BS][BS];
    for (int a = 0; a < BS; ++a)
        for (int c = 0; c < BS; ++c) blk[a][c] = 0.0;
    T* J = (T*)d->J;
    const int64_t Nn = d->Nnode;
    if (valid) {
        const double* __restrict__ rec = d->rec;
        const int64_t Np = d->Np;
        int clo[3] = {0, 0, 0}, chi[3] = {0, 0, 0};
        for (int a = 0; a < DIM; ++a) {
            clo[a] = max(max(n[a], k[a]) - (SHAPE ? 2 : 1), 0);
            chi[a] = min(min(n[a], k[a]) + (SHAPE ? 1 : 0), d->nc[a] - 1);
        }
        for (int cz = (DIM == 3 ? clo[2] : 0); cz <= (DIM == 3 ? chi[2] : 0); ++cz)
            for (int cy = clo[1]; cy <= chi[1]; ++cy) {
                if (clo[0] > chi[0]) continue;
                int64_t rowc = (int64_t)d->nc[0] * (cy + (int64_t)d->nc[1] * cz);
                int p0 = d->cstart[rowc + clo[0]], p1 = d->cstart[rowc + chi[0] + 1];
                for (int p = p0; p < p1; ++p) {
                    int li[3] = {0, 0, 0}, lk[3] = {0, 0, 0};
                    bool in = true;
                    for (int a = 0; a < DIM; ++a) {
                        int bse = d->rbase[a * Np + p];
                        li[a] = n[a] - bse;
                        lk[a] = k[a] - bse;
                        if (li[a] < 0 || li[a] >= WB || lk[a] < 0 || lk[a] >= WB) in = false;
                    }
                    if (!in) continue;
                    double Si, Sk, Gi[DIM], Gk[DIM], s0i, s0k;
                    rec_basis<DIM, WB>(rec, Np, p, li, Si, Gi, s0i);
                    rec_basis<DIM, WB>(rec, Np, p, lk, Sk, Gk, s0k);
                    double fi[DIM * DIM];
                    for (int e = 0; e < DIM * DIM; ++e) fi[e] = rec[(L::FI_ + e) * Np + p];
                    double gi[DIM], gk[DIM];
                    for (int a = 0; a < DIM; ++a) {
                        double t1 = 0.0, t2 = 0.0;
                        for (int c = 0; c < DIM; ++c) {
                            t1 += fi[c * DIM + a] * Gi[c];
                            t2 += fi[c * DIM + a] * Gk[c];
                        }
                        gi[a] = t1;
                        gk[a] = t2;
                    }
                    // displacement-displacement block
                    const double cm = rec[L::CM_ * Np + p];
                    for (int a = 0; a < DIM; ++a)
                        for (int c = 0; c < DIM; ++c) {
                            double t = 0.0;
                            for (int bb = 0; bb < DIM; ++bb) {
                                double u = 0.0;
                                for (int e = 0; e < DIM; ++e)
                                    u += rec[(L::AB_ + ((a * DIM + bb) * DIM + c) * DIM + e) * Np + p] * gk[e];
                                t += gi[bb] * u;
                            }
                            if (a == c) t -= cm * Si * Sk;
                            blk[a][c] += t;
                        }
                    // displacement-pressure
                    const double dvp = rec[L::DV_ * Np + p];
                    for (int a = 0; a < DIM; ++a) blk[a][DIM] += dvp * Sk * gi[a];
                    // pressure-displacement
                    const double bv = rec[L::BV_ * Np + p], dk = rec[L::DK_ * Np + p], ee = rec[L::EE_ * Np + p];
                    double qw[DIM], gpv[DIM];
                    for (int a = 0; a < DIM; ++a) {
                        qw[a] = rec[(L::QW_ + a) * Np + p];
                        gpv[a] = rec[(L::GP_ + a) * Np + p];
                    }
                    double giq = 0.0, gkq = 0.0, gik = 0.0;
                    for (int a = 0; a < DIM; ++a) {
                        giq += gi[a] * qw[a];
                        gkq += gk[a] * qw[a];
                        gik += gi[a] * gk[a];
                    }
                    for (int c = 0; c < DIM; ++c) {
                        double lt = 0.0;
                        for (int a = 0; a < DIM; ++a) lt += gk[a] * rec[(L::LV_ + a * DIM + c) * Np + p];
                        blk[DIM][c] += Si * (bv * gk[c] - lt) + dk * (gk[c] * giq - gi[c] * gkq - gik * gpv[c]) +
                                       ee * gi[c] * Sk;
                    }
                    // pressure-pressure with the PPP term
                    double Pii, Pik;
                    if (SHAPE) {
                        Pii = s0i;
                        Pik = s0k;
                    } else {
                        int64_t cid = 0, mul = 1, lin_i = 0, lin_k = 0;
                        for (int a = 0; a < DIM; ++a) {
                            cid += d->rbase[a * Np + p] * mul;
                            mul *= d->nc[a];
                            lin_i += (int64_t)li[a] << a;
                            lin_k += (int64_t)lk[a] << a;
                        }
                        Pii = d->cellpi[cid * (1 << DIM) + lin_i];
                        Pik = d->cellpi[cid * (1 << DIM) + lin_k];
                    }
                    blk[DIM][DIM] += dk * gik + rec[L::TC_ * Np + p] * (Si - Pii) * (Sk - Pik);
                }
            }
    }
    int64_t pni = 0, pnk = 0;
    if (valid) {
        pni = pad_index(d, n[0], n[1], n[2]);
        pnk = pad_index(d, k[0], k[1], k[2]);
    }
    const bool diag = valid && (sidx == (d->S - 1) / 2);
    for (int a = 0; a < BS; ++a)
        for (int c = 0; c < BS; ++c) {
            double v = blk[a][c];
            if (valid) {
                bool fr = d->dfree[pni * BS + a] != 0;
                bool fc = d->dfree[pnk * BS + c] != 0;
                if (!(fr && fc)) v = (diag && a == c) ? 1.0 : 0.0;
            }
            J[((int64_t)(sidx * BS + a) * BS + c) * Nn + tid] = (T)v;
        }
}

// sum of the residual partials of each problem (one block per problem)
__global__ void k_finalize_norms(Batch B) {
    const int q = blockIdx.x;
    const Dev* d = B.d[q];
    __shared__ double sh[2][TPB];
    double a = 0.0, b2 = 0.0;
    const int64_t nblk = (d->Nnode + TPB - 1) / TPB;   // blocks of k_residual for this problem
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
    Batch Bn = make_batch(g.ddev, g.nnode, TPB);
    if (g.dim == 2 && g.shape == 0) {
        PPM_TIMED(KT_RECORDS, st, hipLaunchKernelGGL((k_records<2, 0>), dim3(Bp.pfx[Bp.n]), dim3(TPB), 0, st, Bp));
        PPM_TIMED(KT_RESIDUAL, st, hipLaunchKernelGGL((k_residual<2, 0>), dim3(Bn.pfx[Bn.n]), dim3(TPB), 0, st, Bn));
    } else if (g.dim == 2 && g.shape == 1) {
        PPM_TIMED(KT_RECORDS, st, hipLaunchKernelGGL((k_records<2, 1>), dim3(Bp.pfx[Bp.n]), dim3(TPB), 0, st, Bp));
        PPM_TIMED(KT_RESIDUAL, st, hipLaunchKernelGGL((k_residual<2, 1>), dim3(Bn.pfx[Bn.n]), dim3(TPB), 0, st, Bn));
    } else {
        PPM_TIMED(KT_RECORDS, st, hipLaunchKernelGGL((k_records<3, 0>), dim3(Bp.pfx[Bp.n]), dim3(TPB), 0, st, Bp));
        PPM_TIMED(KT_RESIDUAL, st, hipLaunchKernelGGL((k_residual<3, 0>), dim3(Bn.pfx[Bn.n]), dim3(TPB), 0, st, Bn));
    }
    hipLaunchKernelGGL(k_finalize_norms, dim3(Bn.n), dim3(TPB), 0, st, Bn);
    if (want_J) launch_jacobian(g, st);
}

void launch_jacobian(const Group& g, hipStream_t st) {
    Batch Bn = make_batch(g.ddev, g.nnode, TPB);
    const dim3 gr(Bn.pfx[Bn.n], g.S), tb(TPB);
    if (g.dim == 2 && g.shape == 0) {
        if (g.mixed) PPM_TIMED(KT_JACOBIAN, st, hipLaunchKernelGGL((k_jacobian<2, 0, float>), gr, tb, 0, st, Bn));
        else PPM_TIMED(KT_JACOBIAN, st, hipLaunchKernelGGL((k_jacobian<2, 0, double>), gr, tb, 0, st, Bn));
    } else if (g.dim == 2 && g.shape == 1) {
        if (g.mixed) PPM_TIMED(KT_JACOBIAN, st, hipLaunchKernelGGL((k_jacobian<2, 1, float>), gr, tb, 0, st, Bn));
        else PPM_TIMED(KT_JACOBIAN, st, hipLaunchKernelGGL((k_jacobian<2, 1, double>), gr, tb, 0, st, Bn));
    } else {
        if (g.mixed) PPM_TIMED(KT_JACOBIAN, st, hipLaunchKernelGGL((k_jacobian<3, 0, float>), gr, tb, 0, st, Bn));
        else PPM_TIMED(KT_JACOBIAN, st, hipLaunchKernelGGL((k_jacobian<3, 0, double>), gr, tb, 0, st, Bn));
    }
}

}  // namespace ppm
