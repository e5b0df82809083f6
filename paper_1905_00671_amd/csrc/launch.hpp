// Host-side launch helpers shared by the kernel files and the runtime of libppmpm.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <array>
#include <initializer_list>
#include <vector>

#include "../../include/ppmpm.h"
#include "ppmpm_internal.hpp"

namespace ppm {

// Problems of one kernel variant stepped together, with their per-problem work sizes.
struct Group {
    int dim = 2, shape = 0, mixed = 0, S = 9, b = 3;
    std::vector<const Dev*> ddev;   // device descriptors
    std::vector<int64_t> np, nnode, ncell, ncell1, npadb, npad, ntile, jblk;
    std::vector<std::array<int, 3>> nn3;   // nodes per axis
    std::vector<const Dev*> hdev;          // host copies of the descriptors
};

// Per-kernel timing with HIP events recorded on the launching stream (off unless enabled).
enum KernelId : int { KT_SPMV = 0, KT_JACOBIAN, KT_RECORDS, KT_RESIDUAL, KT_MG0_RESID, KT_P2G, KT_G2P, KT_PERMUTE,
                      KT_RAP, KT_CELLMAT, KT_MG0_S, KT_COUNT };
bool timing_on();
void timing_begin(hipStream_t st, int id, hipEvent_t* a, hipEvent_t* b);
void timing_end(hipStream_t st, hipEvent_t b);

#define PPM_TIMED(id, st, ...)                          \
    do {                                                \
        if (timing_on() && (id) >= 0) {                 \
            hipEvent_t ea_, eb_;                        \
            timing_begin((st), (id), &ea_, &eb_);       \
            __VA_ARGS__;                                \
            timing_end((st), eb_);                      \
        } else {                                        \
            __VA_ARGS__;                                \
        }                                               \
    } while (0)

// Blocks of `tpb` threads covering work[q] items for every problem q.
inline Batch make_batch(const std::vector<const Dev*>& dd, const std::vector<int64_t>& work, int tpb) {
    Batch B{};
    B.n = (int)dd.size();
    B.pfx[0] = 0;
    for (int q = 0; q < B.n; ++q) {
        int64_t nb = (work[q] + tpb - 1) / tpb;
        if (nb < 1) nb = 1;
        B.pfx[q + 1] = B.pfx[q] + (int)nb;
        B.d[q] = dd[q];
    }
    return B;
}

// Exactly blocks[q] blocks for problem q.
inline Batch make_batch_blocks(const std::vector<const Dev*>& dd, const std::vector<int64_t>& blocks) {
    Batch B{};
    B.n = (int)dd.size();
    B.pfx[0] = 0;
    for (int q = 0; q < B.n; ++q) {
        B.pfx[q + 1] = B.pfx[q] + (int)std::max<int64_t>(blocks[q], 1);
        B.d[q] = dd[q];
    }
    return B;
}

// Node tiles of the gather kernels covering a grid of nn nodes per axis.
inline int64_t node_tiles(int dim, const int* nn) {
    if (dim == 2) return (int64_t)((nn[0] + TILE2X - 1) / TILE2X) * ((nn[1] + TILE2Y - 1) / TILE2Y);
    return (int64_t)((nn[0] + TILE3X - 1) / TILE3X) * ((nn[1] + TILE3Y - 1) / TILE3Y) * ((nn[2] + TILE3Z - 1) / TILE3Z);
}

// Blocks of the Jacobian kernel: x-runs of (TPB / 64) * (64 / b^2) nodes, one per (y, z) row.
inline int64_t jacobian_blocks(int dim, const int* nn) {
    const int b = dim + 1, nodes = (TPB / 64) * (64 / (b * b));
    const int64_t runs = (nn[0] + nodes - 1) / nodes;
    return runs * nn[1] * (dim == 3 ? nn[2] : 1);
}

// Blocks of the 3D block-row gather: a wavefront per (64-node x-run, block entry), 16 entries.
inline int64_t jacgather3_blocks(const std::array<int, 3>& nn) {
    const int64_t waves = (int64_t)((nn[0] + 63) / 64) * nn[1] * nn[2] * 16;
    return (waves + TPB / 64 - 1) / (TPB / 64);
}

// Tiles of the multigrid sweeps covering a level of n nodes per axis.
inline int64_t mg_tiles(int dim, const int* n) {
    if (dim == 2) return (int64_t)((n[0] + MGT2X - 1) / MGT2X) * ((n[1] + MGT2Y - 1) / MGT2Y);
    return (int64_t)((n[0] + MGT3X - 1) / MGT3X) * ((n[1] + MGT3Y - 1) / MGT3Y) * ((n[2] + MGT3Z - 1) / MGT3Z);
}

inline Batch make_batch_one_block(const std::vector<const Dev*>& dd) {
    Batch B{};
    B.n = (int)dd.size();
    for (int q = 0; q <= B.n; ++q) B.pfx[q] = q;
    for (int q = 0; q < B.n; ++q) B.d[q] = dd[q];
    return B;
}

// kern_particles.hip
void launch_set_particles(const Dev* dd, int64_t np, const double* x, const double* vol, const double* mass,
                          const double* lp, const double* v0, const double* p0, hipStream_t st);
void launch_get_field(const Dev* dd, int64_t np, int field, int ncomp, double* out, hipStream_t st);
void launch_sort(const Group& g, hipStream_t st);
void launch_bc(const Dev* dd, int64_t nnode, const uint8_t* uf, const double* ui, const uint8_t* pf,
               const double* pv, const double* fe, const double* qe, hipStream_t st);
void launch_p2g(const Group& g, hipStream_t st);
// nodes below the negligible-mass fraction of the largest nodal mass leave the material (after
// launch_p2g)
void launch_cut_light_nodes(const Group& g, hipStream_t st);
// zero pore pressure on the free surface of the problems with Dev::drain set (after launch_p2g)
void launch_drain_surface(const Group& g, hipStream_t st);
// pressure conditions carried by the flagged points (caller order, NULL: none); last of Stage 1
void launch_point_pfix(const Group& g, const std::vector<const uint8_t*>& flag, const std::vector<const double*>& val,
                       hipStream_t st);

// kern_mass.hip
// nodal forces of the point tractions F[q] (caller order, NULL: none) on the sorted points
void launch_point_force(const Group& g, const std::vector<const double*>& F, const std::vector<const double*>& nrm,
                        hipStream_t st);
// consistent-mass mapping of the P2G fields of the problems with Dev::cons set (after
// launch_p2g); synchronizes the stream to check convergence; iters: CG iterations taken
ppmpm_status launch_mass_solve(const Group& g, const std::vector<const Dev*>& host_copies, hipStream_t st, int* iters);
void launch_cell_proj(const Group& g, hipStream_t st);
void launch_g2p(const Group& g, hipStream_t st);

// kern_assemble.hip
void launch_assemble(const Group& g, bool want_J, hipStream_t st);

// kern_assemble.hip
void launch_jacobian(const Group& g, hipStream_t st);
// coarse: rebuild the Galerkin hierarchy (first Newton iteration of a step); otherwise only the
// fine-level inverse diagonals follow the new Jacobian
void launch_precond_setup(const Group& g, const std::vector<const Dev*>& host_copies, bool coarse, hipStream_t st);
void launch_precond_apply(const Group& g, const std::vector<const Dev*>& host_copies, int iy, int iz, hipStream_t st);
void launch_krylov_init(const Group& g, double rtol, int maxit, hipStream_t st);
void launch_krylov_iters(const Group& g, const std::vector<const Dev*>& host_copies, int iters, double rtol,
                         int maxit, hipStream_t st);
// X += s x on the free dofs (s = 1: the Newton update; s < 0 takes back part of the last one)
void launch_krylov_pick(const Group& g, hipStream_t st);
void launch_newton_update(const Group& g, hipStream_t st, double s = 1.0);
void launch_apply_jacobian(const Dev* dd, const Dev* hd, const double* v_nat, double* y_nat, hipStream_t st);
void launch_nodal_out(const Dev* dd, const Dev* hd, int field, double* out, hipStream_t st);
void launch_residual_out(const Dev* dd, const Dev* hd, double* out, hipStream_t st);
void launch_set_state(const Dev* dd, const Dev* hd, const double* U, const double* P, hipStream_t st);

}  // namespace ppm
