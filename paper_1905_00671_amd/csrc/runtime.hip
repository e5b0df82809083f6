// Host runtime and C ABI of libppmpm: workspace layout, problem descriptors, the time step of
// Sec. 3.1 (Stages 1-4) with the Newton loop of Sec. 3.4 driven from the host over a batch of
// problems, and the inspection entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ppmpm.h"
#include "launch.hpp"
#include "ppmpm_internal.hpp"

using namespace ppm;

static thread_local std::string g_err;

// ---------------------------------------------------------------------------------------------
// per-kernel timing: HIP events recorded on the launching stream around instrumented launches
// ---------------------------------------------------------------------------------------------
namespace ppm {
namespace {
struct PendingEv {
    int id;
    hipEvent_t a, b;
};
bool g_timing = false;
std::vector<PendingEv> g_pending;
std::vector<hipEvent_t> g_pool;
int64_t g_count[KT_COUNT] = {};
double g_ms[KT_COUNT] = {};

hipEvent_t pool_get() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

void timing_collect() {
    for (auto& p : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            g_count[p.id] += 1;
            g_ms[p.id] += ms;
        }
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    g_pending.clear();
}
}  // namespace

bool timing_on() { return g_timing; }

void timing_begin(hipStream_t st, int id, hipEvent_t* a, hipEvent_t* b) {
    *a = pool_get();
    *b = pool_get();
    (void)hipEventRecord(*a, st);
    g_pending.push_back({id, *a, *b});
}

void timing_end(hipStream_t st, hipEvent_t b) { (void)hipEventRecord(b, st); }
}  // namespace ppm

static ppmpm_status fail(ppmpm_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define HIPCHK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(PPMPM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct ppmpm_problem {
    Dev h{};                 // host copy of the device descriptor
    Dev* d = nullptr;        // device copy (inside the workspace)
    Dev* hpin = nullptr;     // pinned staging of the descriptor
    double* spin = nullptr;  // pinned: scalars (NSCAL) + flags (as doubles after)
    int* fpin = nullptr;     // pinned flags
    hipStream_t st = nullptr;
    ppmpm_grid grid{};
    ppmpm_material mat{};
    ppmpm_options opt{};
    int64_t np = 0;
    char* ws = nullptr;
    size_t wsb = 0;
    char* io = nullptr;      // staging for host inputs/outputs
    size_t iob = 0;
    bool have_particles = false;
    bool have_jacobian = false;
    int nrec = 0;
    int mass_iters = 0;      // CG iterations of the last consistent-mass mapping
    uint64_t gen = 0;        // creation number (keys the captured Krylov graphs)
};

// ---------------------------------------------------------------------------------------------
// layout
// ---------------------------------------------------------------------------------------------
namespace {

struct Carver {
    char* base;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? (T*)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

int rec_fields(int dim, int shape) {
    int wb = shape ? 3 : 2;
    if (dim == 2) return wb == 3 ? RecLayout<2, 3>::N : RecLayout<2, 2>::N;
    return RecLayout<3, 2>::N;
}

ppmpm_status validate(const ppmpm_grid* g, const ppmpm_options* o, int64_t np) {
    if (!g || !o) return fail(PPMPM_E_INVALID, "null grid or options");
    if (g->dim != 2 && g->dim != 3) return fail(PPMPM_E_INVALID, "dim must be 2 or 3");
    for (int a = 0; a < g->dim; ++a)
        if (g->ncell[a] < 1 || g->ncell[a] > 100000) return fail(PPMPM_E_INVALID, "bad ncell");
    if (!(g->h > 0)) return fail(PPMPM_E_INVALID, "h must be positive");
    if (o->shape == PPMPM_GIMP && g->dim != 2) return fail(PPMPM_E_INVALID, "GIMP is supported in 2D only");
    if (o->shape != PPMPM_LINEAR && o->shape != PPMPM_GIMP) return fail(PPMPM_E_INVALID, "bad shape");
    if (np < 1 || np > (int64_t)1 << 30) return fail(PPMPM_E_INVALID, "bad particle count");
    if (o->dynamic && !(o->beta > 0 && o->gamma > 0)) return fail(PPMPM_E_INVALID, "bad Newmark parameters");
    if (o->schur != 0 && o->schur != 1) return fail(PPMPM_E_INVALID, "schur must be 0 or 1");
    return PPMPM_OK;
}

// Fill sizes/levels of the host descriptor and carve the workspace (base may be null: sizing).
size_t layout(Dev& h, const ppmpm_grid* g, const ppmpm_options* o, int64_t np, char* base, int* nrec_out) {
    const int D = g->dim;
    h.dim = D;
    h.shape = o->shape;
    h.dyn = o->dynamic;
    h.mixed = o->precision == PPMPM_MIXED;
    h.R = o->shape ? 2 : 1;
    h.W = o->shape ? 3 : 2;
    h.b = D + 1;
    int SW = 2 * h.R + 1;
    h.S = D == 2 ? SW * SW : SW * SW * SW;
    h.Np = np;
    h.Ncell = 1;
    h.Nnode = 1;
    h.Npad = 1;
    for (int a = 0; a < 3; ++a) {
        h.nc[a] = a < D ? g->ncell[a] : 1;
        h.nn[a] = a < D ? g->ncell[a] + 1 : 1;
        h.np1[a] = a < D ? h.nn[a] + 2 * h.R : 1;
        h.x0[a] = a < D ? g->origin[a] : 0.0;
        h.hi[a] = a < D ? g->origin[a] + g->h * g->ncell[a] : 0.0;
        h.Ncell *= h.nc[a];
        h.Nnode *= h.nn[a];
        h.Npad *= h.np1[a];
    }
    h.h = g->h;
    // multigrid levels: halve every axis that still has more than three nodes, until the
    // coarsest system is small enough for the dense inverse
    int nl = 0;
    int n[3] = {h.nn[0], h.nn[1], h.nn[2]};
    while (true) {
        MgLevel& L = h.lev[nl];
        int64_t rows = 1, pads = 1;
        for (int a = 0; a < 3; ++a) {
            L.n[a] = n[a];
            L.np[a] = a < D ? n[a] + 2 * h.R : 1;
            L.cz[a] = 0;
            rows *= L.n[a];
            pads *= L.np[a];
        }
        L.nrow = rows;
        L.npad = pads;
        ++nl;
        bool any = false;
        for (int a = 0; a < D; ++a)
            if (n[a] > 3) any = true;
        if (rows * D <= CMAX || !any || nl == MAXLEV) break;
        for (int a = 0; a < D; ++a) {
            L.cz[a] = n[a] > 3;
            if (L.cz[a]) n[a] = (n[a] - 1) / 2 + 1 + ((n[a] - 1) % 2);
        }
    }
    h.nlev = nl;
    h.ltail = nl - 1;
    for (int l = 0; l < nl; ++l)
        if (h.lev[l].nrow <= TAILMAX) {
            h.ltail = l;
            break;
        }
    // the coarsest level is solved by a dense inverse of at most CMAX unknowns
    if (h.lev[nl - 1].nrow * D > CMAX) return 0;
    const size_t TS = h.mixed ? sizeof(float) : sizeof(double);
    const int nrec = rec_fields(D, o->shape);
    if (nrec_out) *nrec_out = nrec;
    Carver c{base};
    c.take<Dev>(1);  // device descriptor first
    h.pc = c.take<double>((size_t)NPF * np);
    h.pw = c.take<double>((size_t)NPF * np);
    h.idc = c.take<int>(np);
    h.idw = c.take<int>(np);
    h.ps = np;
    h.key = c.take<int>(np);
    h.slot = c.take<int>(np);
    h.order = c.take<int>(np);
    h.ccount = c.take<int>(h.Ncell + 1);
    h.cstart = c.take<int>(h.Ncell + 1);
    const int64_t P = h.Npad, bs = h.b;
    h.M = c.take<double>(P);
    h.Pn = c.take<double>(P);
    h.vn = c.take<double>(P * 3);
    h.an = c.take<double>(P * 3);
    h.pdn = c.take<double>(P);
    h.pddn = c.take<double>(P);
    h.Mp = c.take<double>(P);
    h.dfree = c.take<uint8_t>(P * bs);
    h.bcfix = c.take<uint8_t>(P * bs);
    h.bcval = c.take<double>(P * bs);
    h.fext = c.take<double>(P * bs);
    h.X = c.take<double>(P * bs);
    h.Rv = c.take<double>(P * bs);
    h.cellpi = c.take<double>(h.Ncell * (1 << D));
    h.rec = c.take<double>((size_t)nrec * rec_points_padded(np));
    h.J = c.take<char>((size_t)h.S * bs * bs * jrows_padded(h.Nnode) * TS);
    h.Ke = c.take<char>(D == 3 ? (size_t)h.Ncell * 16 * 64 * TS : 0);
    void** kv[10] = {&h.kx, &h.kr, &h.kh, &h.kp, &h.kv, &h.ks, &h.kt, &h.kph, &h.ksh, &h.kxb};
    for (auto* p : kv) *p = c.take<char>((size_t)P * bs * TS);
    h.kbt = c.take<char>((size_t)P * D * TS);
    for (int l = 0; l < nl; ++l) {
        MgLevel& L = h.lev[l];
        if (l > 0) {
            L.A = c.take<char>((size_t)h.S * D * D * L.nrow * TS);
            L.Sm = c.take<char>((size_t)h.S * L.nrow * TS);
        } else {
            L.A = nullptr;
            // level-0 Schur operator of the diagonal-inverse form (the fixed-stress form reads J)
            L.Sm = o->schur == 1 ? c.take<char>((size_t)h.S * L.nrow * TS) : nullptr;
        }
        L.Ad = c.take<char>((size_t)D * D * L.nrow * TS);
        L.Sd = c.take<char>((size_t)L.nrow * TS);
        L.xa = c.take<char>((size_t)L.npad * D * TS);
        L.ra = c.take<char>((size_t)L.npad * D * TS);
        L.ba = c.take<char>((size_t)L.npad * D * TS);
        L.xs = c.take<char>((size_t)L.npad * TS);
        L.rs = c.take<char>((size_t)L.npad * TS);
        L.bsv = c.take<char>((size_t)L.npad * TS);
    }
    const int64_t nA = h.lev[nl - 1].nrow * D, nS = h.lev[nl - 1].nrow;
    h.cinvA = c.take<char>((size_t)std::min<int64_t>(nA * nA, CMAX * CMAX) * TS);
    h.cinvS = c.take<char>((size_t)std::min<int64_t>(nS * nS, CMAX * CMAX) * TS);
    h.cwork = c.take<double>((size_t)CMAX * CMAX);
    int64_t maxrows = std::max<int64_t>(h.Nnode, np);
    h.maxblocks = std::max<int64_t>(std::max<int64_t>((maxrows + TPB - 1) / TPB + 1, node_tiles(D, h.nn)),
                                    spmv_blocks(D, h.Nnode, true));
    h.partial = c.take<double>((size_t)h.maxblocks * 4);
    h.cons = o->consistent_mass ? 1 : 0;
    h.ncol = o->dynamic ? 2 * D + 3 : 1;
    if (h.cons) {
        const int64_t N = h.Nnode;
        h.mrow = c.take<double>((size_t)h.S * N);
        double** mv[6] = {&h.mb, &h.mx, &h.mr, &h.mz, &h.md, &h.mq};
        for (auto* v : mv) *v = c.take<double>((size_t)h.ncol * N);
        h.mheavy = c.take<uint8_t>(N);
        h.mpart = c.take<double>((size_t)h.maxblocks * 3 * MCOL);
        h.mscal = c.take<double>(MCOL * 8 + 8);
    } else {
        h.mrow = h.mb = h.mx = h.mr = h.mz = h.md = h.mq = h.mpart = h.mscal = nullptr;
        h.mheavy = nullptr;
    }
    h.scal = c.take<double>(NSCAL);
    h.flags = c.take<int>(NFLAG);
    return c.off + 256;
}

size_t io_bytes(const Dev& h) {
    const int D = h.dim;
    size_t a = (size_t)h.Np * (3 * D + 3) * sizeof(double);
    size_t b = (size_t)h.Np * 9 * sizeof(double);
    // boundary data (+ point tractions and normals) + state + residual
    size_t c = (size_t)h.Nnode * (D + 1) * 34 + (size_t)h.Np * (D * 16 + 9) + 16384;
    size_t e = (size_t)h.Nnode * (D + 1) * sizeof(double) * 2;
    return std::max(std::max(a, b), std::max(c, e)) + 4096;
}

double stab_tau(const ppmpm_options* o, double lam, double G, double kappa, double h, double dt) {
    if (o->tau_kind == PPMPM_TAU_OFF) return 0.0;
    if (o->tau_kind == PPMPM_TAU_WHITE) return o->tau_scale / (2.0 * G);
    const double Mp = lam + 2.0 * G, cv = Mp * kappa, r = cv * dt / (h * h);
    if (o->tau_kind == PPMPM_TAU_SUN) {
        double t = (1.0 - 3.0 * r) * (1.0 + std::tanh(2.0 - 12.0 * r)) / Mp;
        return o->tau_scale * std::max(t, 0.0);
    }
    // 2 kappa / c_v = 2 / M, also in the limit kappa -> 0
    double t = 2.0 / Mp - (o->beta / o->gamma) * 12.0 * kappa * dt / (h * h);
    return o->tau_scale * std::max(t, 0.0);
}

// Depth of the Schur-block (S) multigrid.  S is a pressure mass term (c_t/K) M_p plus a Darcy
// diffusion term; on level l their ratio is the diffusion number Fo_l = kappa K / (c_t h_l^2)
// (h_l the smallest node spacing of the level).  From the first level with Fo_l < 1 on, the
// operator is mass-dominated and two damped Jacobi sweeps invert it well enough, so the S cycle
// ends there (level 0: no coarse levels at all; V(1,1) only; ltail or more means the full
// hierarchy).  On the 2D footing (Fo_0 = 0.86) ending at level 0 took fewer Krylov iterations
// than one more level with its coarse correction (240 vs 260 over six steps).
// Damping of the block-Jacobi smoother, below 4 / (3 lambda_max(D^-1 A)) (lambda_max near 2 for
// the 2D stencils, 3.2 for the 27-point trilinear one), chosen by Krylov counts: 2D GIMP footing
// 0.5 / 0.55 / 0.6 / 0.7 / 0.8 took 226 / 212 / 207 / 240 / (no convergence) FP64 iterations over
// six steps; the serving stream (small grids, half of them original-MPM consolidation) took more
// iterations with 0.6 everywhere than with 0.7 (351k vs 340k; 347k with this rule), hence 0.7
// for the 9-point stencil; 3D 0.4 / 0.45 / 0.5 took 172 / 164 / 165 over three steps.
double smoother_damping(const Dev& h) {
    if (h.dim == 3) return 0.5;
    return h.R == 2 ? 0.6 : 0.7;
}

int schur_truncation(const Dev& h) {
    // the diagonal-inverse form is a pressure Laplacian in the undrained limit: full hierarchy
    if (h.mg_nsm != 1 || h.schur) return MAXLEV;
    const double kK = h.kappa * h.Kfs / h.ct;
    for (int l = 0; l < h.ltail; ++l) {
        double hmin = 1e300;
        for (int a = 0; a < h.dim; ++a) {
            const double sp = h.h * (double)(h.nn[a] - 1) / (double)(h.lev[l].n[a] - 1);
            hmin = std::min(hmin, sp);
        }
        if (kK / (hmin * hmin) < 1.0) return l;
    }
    return MAXLEV;
}

// The pinned staging copy is read when the copy executes: callers synchronize the stream
// before the next upload of the same problem.
ppmpm_status upload_desc(ppmpm_problem* p, hipStream_t st) {
    *p->hpin = p->h;
    HIPCHK(hipMemcpyAsync(p->d, p->hpin, sizeof(Dev), hipMemcpyHostToDevice, st));
    return PPMPM_OK;
}
ppmpm_status upload_desc(ppmpm_problem* p) { return upload_desc(p, p->st); }

// copy a caller array of `bytes` into device memory: device pointers pass through, host ones
// are staged in the io region at byte offset `off`
const void* to_device(ppmpm_problem* p, const void* src, size_t bytes, int where, size_t& off, hipStream_t st) {
    if (!src) return nullptr;
    if (where == PPMPM_DEVICE) return src;
    off = (off + 255) & ~size_t(255);
    char* dst = p->io + off;
    off += bytes;
    if (hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) != hipSuccess) return nullptr;
    return dst;
}
const void* to_device(ppmpm_problem* p, const void* src, size_t bytes, int where, size_t& off) {
    return to_device(p, src, bytes, where, off, p->st);
}

Group make_group(const std::vector<ppmpm_problem*>& ps) {
    Group g;
    g.dim = ps[0]->h.dim;
    g.shape = ps[0]->h.shape;
    g.mixed = ps[0]->h.mixed;
    g.S = ps[0]->h.S;
    g.b = ps[0]->h.b;
    for (auto* p : ps) {
        g.ddev.push_back(p->d);
        g.np.push_back(p->h.Np);
        g.nnode.push_back(p->h.Nnode);
        g.ncell.push_back(p->h.Ncell);
        g.ncell1.push_back(p->h.Ncell + 1);
        g.npad.push_back(p->h.Npad);
        g.npadb.push_back(p->h.Npad * p->h.b);
        g.ntile.push_back(node_tiles(p->h.dim, p->h.nn));
        g.jblk.push_back(jacobian_blocks(p->h.dim, p->h.nn));
        g.nn3.push_back({p->h.nn[0], p->h.nn[1], p->h.nn[2]});
        g.hdev.push_back(&p->h);
    }
    return g;
}

std::vector<const Dev*> host_copies(const std::vector<ppmpm_problem*>& ps) {
    std::vector<const Dev*> v;
    for (auto* p : ps) v.push_back(&p->h);
    return v;
}

using clk = std::chrono::steady_clock;
double secs(clk::time_point a, clk::time_point b) { return std::chrono::duration<double>(b - a).count(); }

// scalars and error flags of each problem into its pinned staging (asynchronous)
ppmpm_status fetch_scalars(const std::vector<ppmpm_problem*>& ps, hipStream_t st) {
    for (auto* p : ps) {
        HIPCHK(hipMemcpyAsync(p->spin, p->h.scal, sizeof(double) * NSCAL, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(p->fpin, p->h.flags, sizeof(int) * NFLAG, hipMemcpyDeviceToHost, st));
    }
    return PPMPM_OK;
}

ppmpm_status read_scalars(const std::vector<ppmpm_problem*>& ps, hipStream_t st) {
    ppmpm_status s = fetch_scalars(ps, st);
    if (s) return s;
    HIPCHK(hipStreamSynchronize(st));
    return PPMPM_OK;
}

// Stage 1 for a group: descriptor upload (per-step parameters), boundary data, sort, projection
// cells, P2G.  BC staging happens per problem.
ppmpm_status stage1(const std::vector<ppmpm_problem*>& ps, const double* dt, const ppmpm_bc* const* bcs,
                    hipStream_t st) {
    std::vector<const double*> pforce, pnormal, pfixv;
    std::vector<const uint8_t*> pfixp;
    bool any_force = false, any_pfix = false;
    for (size_t i = 0; i < ps.size(); ++i) {
        ppmpm_problem* p = ps[i];
        Dev& h = p->h;
        const ppmpm_options* o = &p->opt;
        double t = dt[i];
        if (!(t > 0)) return fail(PPMPM_E_INVALID, "dt must be positive");
        h.dt = t;
        h.beta = o->beta;
        h.gamma = o->gamma;
        h.ct = o->dynamic ? o->gamma / (o->beta * t) : 1.0 / t;
        h.hc1 = o->dynamic ? 1.0 - o->gamma / o->beta : 0.0;
        h.hc2 = o->dynamic ? (1.0 - 0.5 * o->gamma / o->beta) * t : 0.0;
        h.tau = stab_tau(o, h.lam, h.G, h.kappa, h.h, t);
        h.Kfs = h.lam + 2.0 * h.G / h.dim;
        // inertia factor of the Newmark fixed-stress modulus: 0 / 0.03 / 0.1 / 0.3 / 1 took 805 /
        // 664 / 515 / 430 / 364 FP64 Krylov iterations over four steps of a 16 x 16 undrained
        // dynamic footing and 3771 / 3327 / 2713 / 2028 / 1725 over six steps of config 2
        h.kin = 1.0;
        h.omega = smoother_damping(h);
        h.mg_nsm = std::max(1, o->mg_smooth);
        h.ls_stop = schur_truncation(h);
        ppmpm_status s = upload_desc(p, st);
        if (s) return s;
        HIPCHK(hipMemsetAsync(h.flags, 0, sizeof(int) * NFLAG, st));
        const ppmpm_bc* bc = bcs ? bcs[i] : nullptr;
        size_t off = 0;
        const int64_t nn = h.Nnode;
        const int D = h.dim;
        int where = bc ? bc->where : PPMPM_HOST;
        const uint8_t* uf = bc ? (const uint8_t*)to_device(p, bc->u_fixed, nn * D, where, off, st) : nullptr;
        const double* ui = bc ? (const double*)to_device(p, bc->u_inc, nn * D * 8, where, off, st) : nullptr;
        const uint8_t* pf = bc ? (const uint8_t*)to_device(p, bc->p_fixed, nn, where, off, st) : nullptr;
        const double* pv = bc ? (const double*)to_device(p, bc->p_val, nn * 8, where, off, st) : nullptr;
        const double* fe = bc ? (const double*)to_device(p, bc->f_ext, nn * D * 8, where, off, st) : nullptr;
        const double* qe = bc ? (const double*)to_device(p, bc->q_ext, nn * 8, where, off, st) : nullptr;
        const double* pfo = bc ? (const double*)to_device(p, bc->point_force, p->np * D * 8, where, off, st) : nullptr;
        const double* pno = pfo ? (const double*)to_device(p, bc->point_normal, p->np * D * 8, where, off, st) : nullptr;
        const uint8_t* ppf = bc ? (const uint8_t*)to_device(p, bc->point_p_fixed, p->np, where, off, st) : nullptr;
        const double* ppv = ppf ? (const double*)to_device(p, bc->point_p_val, p->np * 8, where, off, st) : nullptr;
        if (off > p->iob) return fail(PPMPM_E_OOM, "io staging too small");
        launch_bc(p->d, nn, uf, ui, pf, pv, fe, qe, st);
        pforce.push_back(pfo);
        pnormal.push_back(pno);
        pfixp.push_back(ppf);
        pfixv.push_back(ppv);
        any_force |= pfo != nullptr;
        any_pfix |= ppf != nullptr;
    }
    Group g = make_group(ps);
    launch_sort(g, st);
    if (any_force) launch_point_force(g, pforce, pnormal, st);
    if (g.shape == 0) launch_cell_proj(g, st);
    launch_p2g(g, st);
    launch_cut_light_nodes(g, st);
    bool drain = false, cons = false;
    for (const ppmpm_problem* p : ps) {
        drain |= p->h.drain != 0;
        cons |= p->h.cons != 0;
    }
    if (cons) {
        int it = 0;
        ppmpm_status s = launch_mass_solve(g, g.hdev, st, &it);
        if (s) return fail(s, s == PPMPM_E_NEWTON ? "consistent mass mapping did not converge"
                                                  : "consistent mass mapping failed");
        for (ppmpm_problem* p : ps) p->mass_iters = p->h.cons ? it : 0;
    }
    if (drain) launch_drain_surface(g, st);
    if (any_pfix) launch_point_pfix(g, pfixp, pfixv, st);
    return PPMPM_OK;
}

struct NState {
    int phase = 0;  // 0 Newton, 1 converged, 2 failed
    int status = PPMPM_OK;
    double ru0 = 0, rp0 = 0, atol_u = 0, atol_p = 0;
    int halvings = 0;  // times the last Newton update was halved
    bool kfail = false;  // the last Krylov solve ended above its tolerance (breakdown or limit)
    double merit = 0.0;  // max over blocks of |R_b| / max(|R_b^0|, atol_b) at the last accepted iterate
};

// An inexact Krylov solve (FP32 on the mixed path; on the FP64 path a pressure block that the
// Newton test fixes only loosely, as in free-flying undrained bodies) can return a direction
// whose full step inverts a material point or makes the residual non-finite although a shorter
// step would not.  The update is then halved, up to this many times, before the step is
// reported as failed.  Where the oracle's full steps succeed the FP64 path never halves (the
// iterates agree to rounding), so parity is unaffected.
constexpr int MAX_HALVINGS = 4;

constexpr int ST_PENDING = -1;   // statistics slot of a problem not (yet) finished

// Streams for the second and later kernel-variant groups of a batch, so that the groups' work
// overlaps on the device (the first group runs on the caller's stream).  Created on first use
// per device, at the default priority, and kept until the process ends.
hipStream_t aux_stream(size_t k) {
    static std::mutex mu;
    static std::vector<std::vector<hipStream_t>> pool;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)pool.size() <= dev) pool.resize(dev + 1);
    auto& v = pool[dev];
    while (v.size() < k) {
        hipStream_t t = nullptr;
        if (hipStreamCreateWithFlags(&t, hipStreamNonBlocking) != hipSuccess) return nullptr;
        v.push_back(t);
    }
    return v[k - 1];
}

// Problems of one kernel variant and their Newton state during a batched step.
struct GroupRun {
    std::vector<int> idx;                 // batch indices
    std::vector<ppmpm_problem*> ps;
    std::vector<NState> ns;
    hipStream_t st = nullptr;
    double krtol = 1e-8;
    int kmax = 1000, kcheck = 4;
    // current Newton iteration
    std::vector<ppmpm_problem*> act, cont;
    std::vector<int> actk, contk;
    bool kdone = true;
    int kiters = 0;
};

// ---------------------------------------------------------------------------------------------
// Krylov iterations replayed from captured HIP graphs
// ---------------------------------------------------------------------------------------------
// A chunk of krylov_check BiCGStab iterations is about 40 dependent kernel launches per
// iteration, most of them short on small grids.  The chunk is captured once per (problems, their
// multigrid shapes, iteration count, tolerance, limit) and then replayed: the kernels read every
// scalar from the device and skip their work once a problem has converged, and the chunk holds
// no memory set, copy, event or wait, so a replay is the work of the launches.  Capture runs on a
// private stream (the caller's may be the legacy default stream, which cannot be captured) and
// the graph is launched on the group's stream.  Not used while kernel timing is on (it records
// events around launches); any capture error falls back to direct launches.
struct KGraph {
    std::vector<uint64_t> key;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
};
std::mutex g_kg_mu;
std::vector<KGraph> g_kg;
uint64_t g_kg_clock = 0;
constexpr size_t KG_MAX = 32;

hipStream_t capture_stream() {
    static std::mutex mu;
    static std::vector<std::pair<int, hipStream_t>> streams;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    for (auto& e : streams)
        if (e.first == dev) return e.second;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    streams.push_back({dev, s});
    return s;
}

// drops the graphs that replay work of problem p (before it is destroyed)
void forget_graphs(const ppmpm_problem* p) {
    std::lock_guard<std::mutex> lk(g_kg_mu);
    for (size_t i = 0; i < g_kg.size();) {
        bool hit = false;
        for (size_t j = 0; j + 1 < g_kg[i].key.size(); j += 6)
            if (g_kg[i].key[j] == p->gen) hit = true;
        if (hit) {
            (void)hipGraphExecDestroy(g_kg[i].exec);
            g_kg.erase(g_kg.begin() + i);
        } else {
            ++i;
        }
    }
}

void krylov_chunk(const std::vector<ppmpm_problem*>& cont, int iters, double rtol, int maxit, hipStream_t st) {
    Group gr = make_group(cont);
    const std::vector<const Dev*> hc = host_copies(cont);
    if (ppm::g_timing) {
        launch_krylov_iters(gr, hc, iters, rtol, maxit, st);
        return;
    }
    std::vector<uint64_t> key;
    for (const ppmpm_problem* p : cont) {
        key.push_back(p->gen);
        key.push_back((uint64_t)p->h.nlev);
        key.push_back((uint64_t)p->h.ltail);
        key.push_back((uint64_t)p->h.ls_stop);
        key.push_back((uint64_t)p->h.mg_nsm);
        key.push_back((uint64_t)(uintptr_t)p->d);
    }
    uint64_t rb;
    std::memcpy(&rb, &rtol, sizeof(rb));
    key.push_back((uint64_t)iters);
    key.push_back(rb);
    key.push_back((uint64_t)maxit);
    hipGraphExec_t exec = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_kg_mu);
        for (auto& e : g_kg)
            if (e.key == key) {
                e.used = ++g_kg_clock;
                exec = e.exec;
                break;
            }
    }
    if (!exec) {
        hipStream_t cs = capture_stream();
        hipGraph_t graph = nullptr;
        bool ok = cs && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            launch_krylov_iters(gr, hc, iters, rtol, maxit, cs);
            ok = hipStreamEndCapture(cs, &graph) == hipSuccess && graph;
        }
        if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) (void)hipGraphDestroy(graph);
        if (!ok) {
            (void)hipGetLastError();
            exec = nullptr;
            launch_krylov_iters(gr, hc, iters, rtol, maxit, st);
            return;
        }
        std::lock_guard<std::mutex> lk(g_kg_mu);
        if (g_kg.size() >= KG_MAX) {
            size_t lru = 0;
            for (size_t i = 1; i < g_kg.size(); ++i)
                if (g_kg[i].used < g_kg[lru].used) lru = i;
            (void)hipGraphExecDestroy(g_kg[lru].exec);
            g_kg.erase(g_kg.begin() + lru);
        }
        g_kg.push_back(KGraph{key, exec, ++g_kg_clock});
    }
    if (hipGraphLaunch(exec, st) != hipSuccess) {
        (void)hipGetLastError();
        launch_krylov_iters(gr, hc, iters, rtol, maxit, st);
    }
}

// The batched step.  Problems are grouped by kernel variant (dimension, basis, precision) and
// Krylov options, at most MAXB per group; all groups advance through the stages in lockstep,
// each on its own stream, with one host wait per stage for all of them.  S[i].status is set for
// every problem the step finishes; a returned error leaves the others at ST_PENDING.
ppmpm_status batched_body(ppmpm_problem* const* probs, int nprob, const double* dt, const ppmpm_bc* const* bcs,
                          std::vector<ppmpm_step_stats>& S) {
    // per-problem validation: an invalid problem does not stop the others
    int lead = -1;
    std::vector<int> valid;
    for (int i = 0; i < nprob; ++i) {
        ppmpm_problem* p = probs[i];
        if (!p || !p->have_particles) {
            S[i].status = PPMPM_E_INVALID;
            g_err = "problem without particles";
            continue;
        }
        if (!(dt[i] > 0)) {
            S[i].status = PPMPM_E_INVALID;
            g_err = "dt must be positive";
            continue;
        }
        if (lead < 0) lead = i;
        if (p->st != probs[lead]->st) {
            S[i].status = PPMPM_E_INVALID;
            g_err = "problems of a batch must share one stream";
            continue;
        }
        valid.push_back(i);
    }
    if (valid.empty()) return PPMPM_OK;
    hipStream_t st0 = probs[lead]->st;
    const bool phase_sync = ppm::g_timing;   // exact phase clocks only while kernel timing is on
    auto t0 = clk::now();
    // group by kernel variant and Krylov options
    std::vector<GroupRun> G;
    {
        std::vector<int> used(nprob, 0);
        for (int i : valid) {
            if (used[i]) continue;
            GroupRun g;
            const ppmpm_problem* a = probs[i];
            for (int j : valid) {
                if (used[j] || (int)g.idx.size() >= MAXB) continue;
                const ppmpm_problem* b = probs[j];
                if (a->h.dim == b->h.dim && a->h.shape == b->h.shape && a->h.mixed == b->h.mixed &&
                    a->opt.krylov_rtol == b->opt.krylov_rtol && a->opt.krylov_max == b->opt.krylov_max &&
                    a->opt.krylov_check == b->opt.krylov_check) {
                    g.idx.push_back(j);
                    g.ps.push_back(probs[j]);
                    used[j] = 1;
                }
            }
            g.ns.resize(g.ps.size());
            g.krtol = a->opt.krylov_rtol;
            if (a->h.mixed) g.krtol = std::max(g.krtol, 1e-6);   // FP32 floor; Newton refines
            g.kmax = a->opt.krylov_max;
            g.kcheck = std::max(1, a->opt.krylov_check);
            G.push_back(std::move(g));
        }
    }
    // streams: the first group on the caller's, the others on auxiliary streams joined to it
    hipEvent_t ev_in = nullptr;
    if (G.size() > 1) {
        HIPCHK(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
        HIPCHK(hipEventRecord(ev_in, st0));
    }
    for (size_t k = 0; k < G.size(); ++k) {
        G[k].st = k == 0 ? st0 : aux_stream(k);   // the caller's stream may be the null stream
        if (k > 0 && !G[k].st) return fail(PPMPM_E_DEVICE, "could not create a stream for a kernel-variant group");
        if (k > 0) HIPCHK(hipStreamWaitEvent(G[k].st, ev_in, 0));
    }
    if (ev_in) HIPCHK(hipEventDestroy(ev_in));
    // Stage 1 for every group, then one wait
    auto ta = clk::now();
    for (auto& g : G) {
        std::vector<double> dts;
        std::vector<const ppmpm_bc*> bcv;
        for (int i : g.idx) {
            dts.push_back(dt[i]);
            bcv.push_back(bcs ? bcs[i] : nullptr);
        }
        ppmpm_status s = stage1(g.ps, dts.data(), bcv.data(), g.st);
        if (s) return s;
        HIPCHK(hipGetLastError());
    }
    for (auto& g : G) HIPCHK(hipStreamSynchronize(g.st));
    auto tb = clk::now();
    for (auto& g : G)
        for (size_t k = 0; k < g.ps.size(); ++k) {
            const Dev& h = g.ps[k]->h;
            const ppmpm_options& o = g.ps[k]->opt;
            g.ns[k].atol_u = o.newton_atol_u > 0 ? o.newton_atol_u : 1e-12 * g.ps[k]->mat.E * std::pow(h.h, h.dim - 1);
            g.ns[k].atol_p = o.newton_atol_p > 0 ? o.newton_atol_p : 1e-12 * std::pow(h.h, h.dim) / h.dt;
            S[g.idx[k]].t_sort = secs(ta, tb);
        }
    for (int it = 0;; ++it) {
        // residual of every active problem
        auto t1 = clk::now();
        bool any = false;
        for (auto& g : G) {
            g.act.clear();
            g.actk.clear();
            for (size_t k = 0; k < g.ps.size(); ++k)
                if (g.ns[k].phase == 0) {
                    g.act.push_back(g.ps[k]);
                    g.actk.push_back((int)k);
                }
            if (g.act.empty()) continue;
            any = true;
            Group ga = make_group(g.act);
            launch_assemble(ga, false, g.st);
            HIPCHK(hipGetLastError());
            ppmpm_status s = fetch_scalars(g.act, g.st);
            if (s) return s;
        }
        if (!any) break;
        for (auto& g : G)
            if (!g.act.empty()) HIPCHK(hipStreamSynchronize(g.st));
        auto t2 = clk::now();
        // convergence test (eq. newton-tolerance per residual block), then Jacobian and
        // preconditioner of the problems that continue
        bool anycont = false;
        for (auto& g : G) {
            std::vector<ppmpm_problem*> retry;
            g.cont.clear();
            g.contk.clear();
            for (size_t j = 0; j < g.act.size(); ++j) {
                const int k = g.actk[j];
                ppmpm_problem* p = g.act[j];
                ppmpm_step_stats& so = S[g.idx[k]];
                so.t_assemble += secs(t1, t2);
                const double ru = std::sqrt(p->spin[SC_RU2]), rp = std::sqrt(p->spin[SC_RP2]);
                if (it < PPMPM_MAX_HIST) {
                    so.res_u[it] = ru;
                    so.res_p[it] = rp;
                }
                so.newton_iters = it;
                if (p->fpin[FL_INVERTED] || p->fpin[FL_NONFINITE] || !std::isfinite(ru) || !std::isfinite(rp)) {
                    if (it > 0 && g.ns[k].halvings < MAX_HALVINGS) {
                        // take back half of what remains of the last update, clear the flags and
                        // evaluate the residual again in the next pass
                        g.ns[k].halvings++;
                        retry.push_back(p);
                        continue;
                    }
                    g.ns[k].phase = 2;
                    g.ns[k].status = PPMPM_E_NONFINITE;
                    continue;
                }
                if (it > 0 && g.ns[k].kfail && g.ns[k].halvings < MAX_HALVINGS) {
                    // the direction came from a linear solve that did not converge: accept it
                    // only if it lowers the residual, else take back half of it
                    const double m = std::max(ru / std::max(g.ns[k].ru0, g.ns[k].atol_u),
                                              rp / std::max(g.ns[k].rp0, g.ns[k].atol_p));
                    if (!(m < g.ns[k].merit)) {
                        g.ns[k].halvings++;
                        retry.push_back(p);
                        continue;
                    }
                }
                g.ns[k].halvings = 0;
                if (p->fpin[FL_BOUNDS]) {
                    g.ns[k].phase = 2;
                    g.ns[k].status = PPMPM_E_DEVICE;
                    continue;
                }
                if (it == 0) {
                    g.ns[k].ru0 = ru;
                    g.ns[k].rp0 = rp;
                }
                g.ns[k].merit = std::max(ru / std::max(g.ns[k].ru0, g.ns[k].atol_u),
                                         rp / std::max(g.ns[k].rp0, g.ns[k].atol_p));
                const double rt = p->opt.newton_rtol;
                const bool cu = ru <= std::max(rt * g.ns[k].ru0, g.ns[k].atol_u);
                const bool cp = rp <= std::max(rt * g.ns[k].rp0, g.ns[k].atol_p);
                if (cu && cp) {
                    g.ns[k].phase = 1;
                    so.converged = 1;
                    continue;
                }
                if (it >= p->opt.newton_max) {
                    g.ns[k].phase = 2;
                    g.ns[k].status = PPMPM_E_NEWTON;
                    continue;
                }
                g.cont.push_back(p);
                g.contk.push_back(k);
            }
            for (auto* p : retry) {
                int k = 0;
                while (g.ps[k] != p) ++k;
                const double s = -std::ldexp(1.0, -g.ns[k].halvings);   // -1/2, -1/4, ...
                launch_newton_update(make_group({p}), g.st, s);
                HIPCHK(hipMemsetAsync(p->h.flags, 0, sizeof(int) * NFLAG, g.st));
            }
            if (g.cont.empty()) continue;
            anycont = true;
            Group gc = make_group(g.cont);
            launch_jacobian(gc, g.st);
            launch_precond_setup(gc, host_copies(g.cont), it == 0, g.st);
            HIPCHK(hipGetLastError());
        }
        if (!anycont) continue;
        auto t3 = clk::now();
        if (phase_sync)
            for (auto& g : G)
                if (!g.cont.empty()) HIPCHK(hipStreamSynchronize(g.st));
        auto t4 = clk::now();
        // Krylov solves: every group advances krylov_check iterations, then one wait
        for (auto& g : G) {
            g.kdone = g.cont.empty();
            g.kiters = 0;
            if (g.kdone) continue;
            launch_krylov_init(make_group(g.cont), g.krtol, g.kmax, g.st);
        }
        while (true) {
            bool pending = false;
            for (auto& g : G) {
                if (g.kdone) continue;
                krylov_chunk(g.cont, g.kcheck, g.krtol, g.kmax, g.st);
                HIPCHK(hipGetLastError());
                ppmpm_status s = fetch_scalars(g.cont, g.st);
                if (s) return s;
                g.kiters += g.kcheck;
                pending = true;
            }
            if (!pending) break;
            for (auto& g : G) {
                if (g.kdone) continue;
                HIPCHK(hipStreamSynchronize(g.st));
                bool all = true;
                for (auto* p : g.cont)
                    if (p->spin[SC_DONE] == 0.0) all = false;
                if (all || g.kiters >= g.kmax) g.kdone = true;
            }
        }
        for (auto& g : G)
            if (!g.cont.empty()) {
                Group gc = make_group(g.cont);
                launch_krylov_pick(gc, g.st);
                launch_newton_update(gc, g.st);
            }
        HIPCHK(hipGetLastError());
        if (phase_sync)
            for (auto& g : G)
                if (!g.cont.empty()) HIPCHK(hipStreamSynchronize(g.st));
        auto t5 = clk::now();
        for (auto& g : G)
            for (size_t j = 0; j < g.cont.size(); ++j) {
                ppmpm_step_stats& so = S[g.idx[g.contk[j]]];
                const int kit = (int)g.cont[j]->spin[SC_ITER];
                if (it < PPMPM_MAX_HIST) so.krylov_iters[it] = kit;
                so.krylov_total += kit;
                // breakdowns: those restarted from the current residual, and a final one
                so.krylov_breakdowns += (int)g.cont[j]->spin[SC_NRESTART] + (g.cont[j]->spin[SC_BREAK] != 0.0 ? 1 : 0);
                g.ns[g.contk[j]].kfail = !(g.cont[j]->spin[SC_RR] <= g.cont[j]->spin[SC_TOL2]);
                so.t_precond += phase_sync ? secs(t3, t4) : 0.0;
                so.t_krylov += phase_sync ? secs(t4, t5) : secs(t2, t5);
            }
    }
    // Stages 3-4 for the converged problems
    auto t6 = clk::now();
    std::vector<std::vector<ppmpm_problem*>> okp(G.size());
    std::vector<std::vector<int>> okk(G.size());
    for (size_t gi = 0; gi < G.size(); ++gi) {
        GroupRun& g = G[gi];
        for (size_t k = 0; k < g.ps.size(); ++k)
            if (g.ns[k].phase == 1) {
                okp[gi].push_back(g.ps[k]);
                okk[gi].push_back((int)k);
            }
        if (okp[gi].empty()) continue;
        launch_g2p(make_group(okp[gi]), g.st);
        HIPCHK(hipGetLastError());
        ppmpm_status s = fetch_scalars(okp[gi], g.st);
        if (s) return s;
    }
    for (size_t gi = 0; gi < G.size(); ++gi) {
        GroupRun& g = G[gi];
        if (okp[gi].empty()) continue;
        HIPCHK(hipStreamSynchronize(g.st));
        for (size_t j = 0; j < okp[gi].size(); ++j) {
            ppmpm_problem* p = okp[gi][j];
            const int k = okk[gi][j];
            if (p->fpin[FL_INVERTED]) {
                g.ns[k].status = PPMPM_E_NONFINITE;
                continue;
            }
            if (p->fpin[FL_OUTSIDE]) {
                g.ns[k].status = PPMPM_E_OUT_OF_GRID;
                continue;
            }
            // commit: the working buffer becomes the state
            std::swap(p->h.pc, p->h.pw);
            std::swap(p->h.idc, p->h.idw);
            ppmpm_status s = upload_desc(p, g.st);
            if (s) return s;
        }
    }
    // the descriptor uploads complete before the pinned staging is reused; the caller's stream
    // waits for every group
    for (size_t gi = 0; gi < G.size(); ++gi) HIPCHK(hipStreamSynchronize(G[gi].st));
    if (ppm::g_timing) ppm::timing_collect();
    auto t7 = clk::now();
    for (auto& g : G)
        for (size_t k = 0; k < g.ps.size(); ++k) {
            ppmpm_step_stats& so = S[g.idx[k]];
            so.t_g2p = secs(t6, t7);
            so.status = g.ns[k].status;
            so.ngrid_levels = g.ps[k]->h.nlev;
            so.mass_iters = g.ps[k]->mass_iters;
            so.t_total = secs(t0, t7);
        }
    return PPMPM_OK;
}

}  // namespace

static ppmpm_status init_problem(ppmpm_problem* p, const ppmpm_grid* grid, const ppmpm_material* mat,
                                 const ppmpm_options* opt, void* workspace, size_t ws_bytes, void* hip_stream,
                                 int64_t np);

// ---------------------------------------------------------------------------------------------
// Workspace in a file-scope device array, for the entry point whose callers cannot allocate
// (code under stream capture, serving loops and harnesses that forbid hipMalloc).  Each device
// holds its own copy of `scratch` until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns for the current device (taken once per device).
// ---------------------------------------------------------------------------------------------
constexpr size_t STATIC_WS_BYTES = (size_t)64 << 20;
constexpr int STATIC_MAX_DEVICES = 64;
static __device__ __align__(256) char scratch[STATIC_WS_BYTES];

static ppmpm_status scratch_address(void** out) {
    static std::mutex mu;
    static void* ptr[STATIC_MAX_DEVICES] = {};
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= STATIC_MAX_DEVICES) return fail(PPMPM_E_DEVICE, "device index beyond the static workspace table");
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void* a = nullptr;
        hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !a)
            return fail(PPMPM_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        ptr[dev] = a;
    }
    *out = ptr[dev];
    return PPMPM_OK;
}

// ---------------------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------------------
namespace {
// checkpoint header (padded to STATE_HDR bytes)
struct StateHeader {
    char magic[8];
    int32_t version, dim, shape, npf;
    int64_t np;
    int32_t ncell[3], pad;
    double h;
};
constexpr size_t STATE_HDR = 64;
static_assert(sizeof(StateHeader) <= STATE_HDR, "checkpoint header");

StateHeader state_header(const ppmpm_problem* p) {
    StateHeader hd{};
    std::memcpy(hd.magic, "PPMPMST1", 8);
    hd.version = 1;
    hd.dim = p->h.dim;
    hd.shape = p->h.shape;
    hd.npf = NPF;
    hd.np = p->np;
    for (int a = 0; a < 3; ++a) hd.ncell[a] = p->h.nc[a];
    hd.h = p->h.h;
    return hd;
}

size_t state_field_bytes(const ppmpm_problem* p) { return (size_t)NPF * p->np * sizeof(double); }
size_t state_bytes(const ppmpm_problem* p) {
    return STATE_HDR + state_field_bytes(p) + ((size_t)p->np * sizeof(int) + 7) / 8 * 8;
}
}  // namespace

extern "C" {

size_t ppmpm_workspace_bytes(const ppmpm_grid* grid, int64_t np, const ppmpm_options* opt) {
    if (validate(grid, opt, np) != PPMPM_OK) return 0;
    Dev h{};
    size_t core = layout(h, grid, opt, np, nullptr, nullptr);
    if (core == 0) {
        g_err = "grid too elongated: the multigrid cannot coarsen it to a dense coarsest level";
        return 0;
    }
    return core + io_bytes(h) + 256;
}

ppmpm_status ppmpm_create(const ppmpm_grid* grid, const ppmpm_material* mat, const ppmpm_options* opt,
                          void* workspace, size_t ws_bytes, void* hip_stream, int64_t np, ppmpm_problem** out) {
    if (!out) return fail(PPMPM_E_INVALID, "null out");
    *out = nullptr;
    ppmpm_status s = validate(grid, opt, np);
    if (s) return s;
    if (!mat) return fail(PPMPM_E_INVALID, "null material");
    if (mat->model == PPMPM_HENCKY && grid->dim == 3) return fail(PPMPM_E_INVALID, "Hencky is plane strain only");
    if (!(mat->E > 0) || !(mat->nu > -1.0 && mat->nu < 0.5) || !(mat->mu_f > 0) || !(mat->k >= 0))
        return fail(PPMPM_E_INVALID, "bad material constants");
    if (!(mat->phi0 >= 0.0 && mat->phi0 < 1.0)) return fail(PPMPM_E_INVALID, "initial porosity outside [0, 1)");
    if (!(mat->alpha_vis >= 0.0)) return fail(PPMPM_E_INVALID, "negative damping parameter");
    if (((uintptr_t)workspace & 255) != 0) return fail(PPMPM_E_INVALID, "workspace must be 256-byte aligned");
    size_t need = ppmpm_workspace_bytes(grid, np, opt);
    if (need == 0) return PPMPM_E_INVALID;   // message set by ppmpm_workspace_bytes
    if (!workspace || ws_bytes < need) return fail(PPMPM_E_OOM, "workspace smaller than ppmpm_workspace_bytes");
    ppmpm_problem* p = new ppmpm_problem();
    {
        hipError_t e = hipHostMalloc((void**)&p->hpin, sizeof(Dev));
        if (e == hipSuccess) e = hipHostMalloc((void**)&p->spin, sizeof(double) * NSCAL);
        if (e == hipSuccess) e = hipHostMalloc((void**)&p->fpin, sizeof(int) * NFLAG);
        if (e != hipSuccess) {
            ppmpm_destroy(p);
            return fail(PPMPM_E_DEVICE, std::string("pinned host allocation failed: ") + hipGetErrorString(e));
        }
    }
    s = init_problem(p, grid, mat, opt, workspace, ws_bytes, hip_stream, np);
    if (s) {
        ppmpm_destroy(p);
        return s;
    }
    *out = p;
    return PPMPM_OK;
}

// Fills a problem whose staging buffers (hpin, spin, fpin) are set: descriptor, workspace layout,
// cleared workspace, uploaded descriptor.  Allocates nothing.
static ppmpm_status init_problem(ppmpm_problem* p, const ppmpm_grid* grid, const ppmpm_material* mat,
                                 const ppmpm_options* opt, void* workspace, size_t ws_bytes, void* hip_stream,
                                 int64_t np) {
    static std::atomic<uint64_t> generation{0};
    p->gen = ++generation;
    p->grid = *grid;
    p->mat = *mat;
    p->opt = *opt;
    if (p->opt.newton_max <= 0) p->opt.newton_max = 25;
    if (p->opt.krylov_max <= 0) p->opt.krylov_max = 1000;
    if (p->opt.krylov_check <= 0) p->opt.krylov_check = 4;
    if (!(p->opt.newton_rtol > 0)) p->opt.newton_rtol = 1e-8;
    if (!(p->opt.krylov_rtol > 0)) p->opt.krylov_rtol = 1e-8;
    p->np = np;
    p->ws = (char*)workspace;
    p->wsb = ws_bytes;
    p->st = (hipStream_t)hip_stream;
    size_t used = layout(p->h, grid, opt, np, p->ws, &p->nrec);
    p->d = (Dev*)p->ws;
    p->io = p->ws + ((used + 255) & ~size_t(255));
    p->iob = ws_bytes - (size_t)(p->io - p->ws);
    Dev& h = p->h;
    h.model = mat->model;
    h.lam = mat->E * mat->nu / ((1.0 + mat->nu) * (1.0 - 2.0 * mat->nu));
    h.G = mat->E / (2.0 * (1.0 + mat->nu));
    h.kappa = mat->k / mat->mu_f;
    h.phi0 = mat->phi0;
    h.alpha_vis = opt->dynamic ? mat->alpha_vis : 0.0;   // quasi-static: no viscous stress
    h.drain = opt->drained_surface ? 1 : 0;
    h.negl = opt->negligible_mass > 0.0 ? opt->negligible_mass : NEGLIGIBLE_MASS;
    h.schur = opt->schur;
    h.rho_f = mat->rho_f;
    for (int a = 0; a < 3; ++a) h.g[a] = a < grid->dim ? mat->g[a] : 0.0;
    h.dt = 1.0;
    h.beta = opt->beta;
    h.gamma = opt->gamma;
    h.omega = smoother_damping(h);
    h.mg_nsm = std::max(1, opt->mg_smooth);
    h.ls_stop = MAXLEV;
    HIPCHK(hipMemsetAsync(p->ws, 0, used, p->st));
    return upload_desc(p);
}

ppmpm_status ppmpm_set_particles(ppmpm_problem* p, int64_t np, const double* x, const double* vol, const double* mass,
                                 const double* lp, const double* v0, const double* p0, int where) {
    if (!p || np != p->np || !x || !vol || !mass) return fail(PPMPM_E_INVALID, "bad set_particles arguments");
    const int D = p->h.dim;
    size_t off = 0;
    const double* dx = (const double*)to_device(p, x, np * D * 8, where, off);
    const double* dvol = (const double*)to_device(p, vol, np * 8, where, off);
    const double* dm = (const double*)to_device(p, mass, np * 8, where, off);
    const double* dlp = (const double*)to_device(p, lp, np * D * 8, where, off);
    const double* dv0 = (const double*)to_device(p, v0, np * D * 8, where, off);
    const double* dp0 = (const double*)to_device(p, p0, np * 8, where, off);
    if (off > p->iob) return fail(PPMPM_E_OOM, "io staging too small");
    HIPCHK(hipMemsetAsync(p->h.flags, 0, sizeof(int) * NFLAG, p->st));
    launch_set_particles(p->d, np, dx, dvol, dm, dlp, dv0, dp0, p->st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(p->fpin, p->h.flags, sizeof(int) * NFLAG, hipMemcpyDeviceToHost, p->st));
    HIPCHK(hipStreamSynchronize(p->st));
    if (p->fpin[FL_OUTSIDE]) return fail(PPMPM_E_OUT_OF_GRID, "a material point lies outside the grid (or lp > h/2)");
    p->have_particles = true;
    return PPMPM_OK;
}

ppmpm_status ppmpm_step_batched(ppmpm_problem* const* probs, int nprob, const double* dt, const ppmpm_bc* const* bcs,
                                ppmpm_step_stats* stats) {
    if (!probs || nprob < 1 || !dt) return fail(PPMPM_E_INVALID, "bad batch");
    std::vector<ppmpm_step_stats> S(nprob);
    for (auto& so : S) {
        std::memset(&so, 0, sizeof(so));
        so.status = ST_PENDING;
    }
    ppmpm_status s = batched_body(probs, nprob, dt, bcs, S);
    // every problem gets a status: those the body did not finish share its failure
    ppmpm_status first_err = s;
    for (int i = 0; i < nprob; ++i) {
        if (S[i].status == ST_PENDING) S[i].status = s != PPMPM_OK ? s : PPMPM_E_DEVICE;
        if (S[i].status != PPMPM_OK && first_err == PPMPM_OK) first_err = (ppmpm_status)S[i].status;
        if (stats) stats[i] = S[i];
    }
    if (first_err != PPMPM_OK && s == PPMPM_OK) {
        const char* names[] = {"ok", "invalid", "oom", "device", "Newton did not converge", "krylov",
                               "non-finite residual or inverted material point", "material point left the grid"};
        g_err = std::string("step failed: ") + names[first_err];
    }
    return first_err;
}

ppmpm_status ppmpm_step(ppmpm_problem* p, double dt, const ppmpm_bc* bc, ppmpm_step_stats* stats) {
    ppmpm_problem* probs[1] = {p};
    const ppmpm_bc* bcs[1] = {bc};
    return ppmpm_step_batched(probs, 1, &dt, bcs, stats);
}

ppmpm_status ppmpm_get_field(const ppmpm_problem* pc, int field, double* out, int where) {
    ppmpm_problem* p = const_cast<ppmpm_problem*>(pc);
    if (!p || !out || field < 0 || field > 10) return fail(PPMPM_E_INVALID, "bad get_field arguments");
    const int D = p->h.dim;
    int ncomp = 1;
    switch (field) {
        case PPMPM_FIELD_X: case PPMPM_FIELD_U: case PPMPM_FIELD_V: case PPMPM_FIELD_A: case PPMPM_FIELD_LP: ncomp = D; break;
        case PPMPM_FIELD_F: ncomp = D * D; break;
        case PPMPM_FIELD_SIG: ncomp = 9; break;
        default: ncomp = 1;
    }
    size_t bytes = (size_t)p->np * ncomp * sizeof(double);
    double* dst = where == PPMPM_DEVICE ? out : (double*)p->io;
    if (where != PPMPM_DEVICE && bytes > p->iob) return fail(PPMPM_E_OOM, "io staging too small");
    launch_get_field(p->d, p->np, field, ncomp, dst, p->st);
    HIPCHK(hipGetLastError());
    if (where != PPMPM_DEVICE) HIPCHK(hipMemcpyAsync(out, dst, bytes, hipMemcpyDeviceToHost, p->st));
    HIPCHK(hipStreamSynchronize(p->st));
    return PPMPM_OK;
}

ppmpm_status ppmpm_state_bytes(const ppmpm_problem* p, size_t* bytes) {
    if (!p || !bytes) return fail(PPMPM_E_INVALID, "bad state_bytes arguments");
    *bytes = state_bytes(p);
    return PPMPM_OK;
}

ppmpm_status ppmpm_save_state(const ppmpm_problem* pc, void* out, size_t bytes, int where) {
    ppmpm_problem* p = const_cast<ppmpm_problem*>(pc);
    if (!p || !out || !p->have_particles || bytes < state_bytes(p)) return fail(PPMPM_E_INVALID, "bad save_state arguments");
    char hbuf[STATE_HDR] = {};
    const StateHeader hd = state_header(p);
    std::memcpy(hbuf, &hd, sizeof(hd));
    char* o = (char*)out;
    const size_t fb = state_field_bytes(p), ib = (size_t)p->np * sizeof(int);
    const hipMemcpyKind k = where == PPMPM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    HIPCHK(hipMemcpyAsync(o + STATE_HDR, p->h.pc, fb, k, p->st));
    HIPCHK(hipMemcpyAsync(o + STATE_HDR + fb, p->h.idc, ib, k, p->st));
    if (where == PPMPM_DEVICE) HIPCHK(hipMemcpyAsync(o, hbuf, STATE_HDR, hipMemcpyHostToDevice, p->st));
    else std::memcpy(o, hbuf, STATE_HDR);
    HIPCHK(hipStreamSynchronize(p->st));   // also keeps hbuf alive until its copy is done
    return PPMPM_OK;
}

ppmpm_status ppmpm_load_state(ppmpm_problem* p, const void* in, size_t bytes, int where) {
    if (!p || !in || bytes < state_bytes(p)) return fail(PPMPM_E_INVALID, "bad load_state arguments");
    char hbuf[STATE_HDR];
    if (where == PPMPM_DEVICE) {
        HIPCHK(hipMemcpyAsync(hbuf, in, STATE_HDR, hipMemcpyDeviceToHost, p->st));
        HIPCHK(hipStreamSynchronize(p->st));
    } else {
        std::memcpy(hbuf, in, STATE_HDR);
    }
    StateHeader hd;
    std::memcpy(&hd, hbuf, sizeof(hd));
    const StateHeader want = state_header(p);
    bool ok = std::memcmp(hd.magic, want.magic, 8) == 0 && hd.version == want.version && hd.dim == want.dim &&
              hd.shape == want.shape && hd.npf == want.npf && hd.np == want.np && hd.h == want.h;
    for (int a = 0; a < 3; ++a) ok = ok && hd.ncell[a] == want.ncell[a];
    if (!ok) return fail(PPMPM_E_INVALID, "checkpoint does not match this problem");
    const char* i = (const char*)in;
    const size_t fb = state_field_bytes(p), ib = (size_t)p->np * sizeof(int);
    const hipMemcpyKind k = where == PPMPM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    HIPCHK(hipMemcpyAsync(p->h.pc, i + STATE_HDR, fb, k, p->st));
    HIPCHK(hipMemcpyAsync(p->h.idc, i + STATE_HDR + fb, ib, k, p->st));
    HIPCHK(hipStreamSynchronize(p->st));
    p->have_particles = true;
    p->have_jacobian = false;
    return PPMPM_OK;
}

ppmpm_status ppmpm_eval_residual(ppmpm_problem* p, double dt, const ppmpm_bc* bc, const double* U, const double* P,
                                 double* R, int where) {
    if (!p || !p->have_particles || !U || !P || !R) return fail(PPMPM_E_INVALID, "bad eval_residual arguments");
    std::vector<ppmpm_problem*> ps{p};
    const ppmpm_bc* bcs[1] = {bc};
    ppmpm_status s = stage1(ps, &dt, bcs, p->st);
    if (s) return s;
    const int64_t nn = p->h.Nnode;
    const int D = p->h.dim;
    // stage1 used the front of the io region for the boundary data; stage the state after it
    size_t off = (size_t)nn * (D + 1) * (2 * sizeof(double) + 2) + 4096;
    if (bc && bc->point_force) off += (size_t)p->np * D * 16 + 512;
    if (bc && bc->point_p_fixed) off += (size_t)p->np * 9 + 512;
    const double* dU = (const double*)to_device(p, U, nn * D * 8, where, off);
    const double* dP = (const double*)to_device(p, P, nn * 8, where, off);
    double* dR = where == PPMPM_DEVICE ? R : (double*)(p->io + ((off + 255) & ~size_t(255)));
    launch_set_state(p->d, &p->h, dU, dP, p->st);
    Group g = make_group(ps);
    launch_assemble(g, true, p->st);
    launch_residual_out(p->d, &p->h, dR, p->st);
    HIPCHK(hipGetLastError());
    if (where != PPMPM_DEVICE) HIPCHK(hipMemcpyAsync(R, dR, nn * (D + 1) * 8, hipMemcpyDeviceToHost, p->st));
    s = read_scalars(ps, p->st);
    if (s) return s;
    p->have_jacobian = true;
    if (p->fpin[FL_INVERTED]) return fail(PPMPM_E_NONFINITE, "inverted material point");
    return PPMPM_OK;
}

ppmpm_status ppmpm_eval_residual_static(const ppmpm_grid* grid, const ppmpm_material* mat, const ppmpm_options* opt,
                                        int64_t np, const double* x, const double* vol, const double* mass,
                                        const double* lp, const double* v0, const double* p0, double dt,
                                        const ppmpm_bc* bc, const double* U, const double* P, double* R,
                                        void* hip_stream, int where) {
    ppmpm_status s = validate(grid, opt, np);
    if (s) return s;
    if (!mat) return fail(PPMPM_E_INVALID, "null material");
    if (mat->model == PPMPM_HENCKY && grid->dim == 3) return fail(PPMPM_E_INVALID, "Hencky is plane strain only");
    if (!(mat->E > 0) || !(mat->nu > -1.0 && mat->nu < 0.5) || !(mat->mu_f > 0) || !(mat->k >= 0))
        return fail(PPMPM_E_INVALID, "bad material constants");
    if (!(mat->phi0 >= 0.0 && mat->phi0 < 1.0)) return fail(PPMPM_E_INVALID, "initial porosity outside [0, 1)");
    if (!(mat->alpha_vis >= 0.0)) return fail(PPMPM_E_INVALID, "negative damping parameter");
    const size_t need = ppmpm_workspace_bytes(grid, np, opt);
    if (need == 0) return PPMPM_E_INVALID;   // message set by ppmpm_workspace_bytes
    if (need > STATIC_WS_BYTES)
        return fail(PPMPM_E_OOM, "problem needs " + std::to_string(need) + " workspace bytes; the static workspace holds " +
                                     std::to_string(STATIC_WS_BYTES));
    void* ws = nullptr;
    s = scratch_address(&ws);
    if (s) return s;
    // host staging of the descriptor and of the scalars: pageable, process-wide (calls that
    // overlap race on them as on the device array); each upload is followed by a stream
    // synchronization before the next one
    static Dev s_desc;
    static double s_scal[NSCAL];
    static int s_flags[NFLAG];
    ppmpm_problem pb;
    pb.hpin = &s_desc;
    pb.spin = s_scal;
    pb.fpin = s_flags;
    s = init_problem(&pb, grid, mat, opt, ws, STATIC_WS_BYTES, hip_stream, np);
    if (s == PPMPM_OK) s = ppmpm_set_particles(&pb, np, x, vol, mass, lp, v0, p0, where);
    if (s == PPMPM_OK) s = ppmpm_eval_residual(&pb, dt, bc, U, P, R, where);
    (void)hipStreamSynchronize(pb.st);
    return s;
}

ppmpm_status ppmpm_apply_jacobian(ppmpm_problem* p, const double* v, double* y, int where) {
    if (!p || !p->have_jacobian || !v || !y) return fail(PPMPM_E_INVALID, "no Jacobian assembled");
    const int64_t n = p->h.Nnode * p->h.b;
    size_t off = 0;
    const double* dv = (const double*)to_device(p, v, n * 8, where, off);
    off = (off + 255) & ~size_t(255);
    double* dy = where == PPMPM_DEVICE ? y : (double*)(p->io + off);
    launch_apply_jacobian(p->d, &p->h, dv, dy, p->st);
    HIPCHK(hipGetLastError());
    if (where != PPMPM_DEVICE) HIPCHK(hipMemcpyAsync(y, dy, n * 8, hipMemcpyDeviceToHost, p->st));
    HIPCHK(hipStreamSynchronize(p->st));
    return PPMPM_OK;
}

ppmpm_status ppmpm_get_nodal(const ppmpm_problem* pc, int field, double* out, int where) {
    ppmpm_problem* p = const_cast<ppmpm_problem*>(pc);
    if (!p || !out || field < 0 || field > 3) return fail(PPMPM_E_INVALID, "bad get_nodal arguments");
    const int64_t n = field >= 2 ? p->h.Nnode * p->h.b : p->h.Nnode;
    double* dst = where == PPMPM_DEVICE ? out : (double*)p->io;
    launch_nodal_out(p->d, &p->h, field, dst, p->st);
    HIPCHK(hipGetLastError());
    if (where != PPMPM_DEVICE) HIPCHK(hipMemcpyAsync(out, dst, n * 8, hipMemcpyDeviceToHost, p->st));
    HIPCHK(hipStreamSynchronize(p->st));
    return PPMPM_OK;
}

ppmpm_status ppmpm_destroy(ppmpm_problem* p) {
    if (!p) return PPMPM_OK;
    if (p->st) (void)hipStreamSynchronize(p->st);
    forget_graphs(p);
    if (p->hpin) (void)hipHostFree(p->hpin);
    if (p->spin) (void)hipHostFree(p->spin);
    if (p->fpin) (void)hipHostFree(p->fpin);
    delete p;
    return PPMPM_OK;
}

const char* ppmpm_last_error(void) { return g_err.c_str(); }

ppmpm_status ppmpm_timing_enable(int on) {
    ppm::timing_collect();
    ppm::g_timing = on != 0;
    return PPMPM_OK;
}

ppmpm_status ppmpm_timing_reset(void) {
    ppm::timing_collect();
    for (int i = 0; i < KT_COUNT; ++i) {
        ppm::g_count[i] = 0;
        ppm::g_ms[i] = 0.0;
    }
    return PPMPM_OK;
}

ppmpm_status ppmpm_timing_get(int kernel, int64_t* launches, double* total_ms) {
    if (kernel < 0 || kernel >= KT_COUNT || !launches || !total_ms) return fail(PPMPM_E_INVALID, "bad kernel id");
    ppm::timing_collect();
    *launches = ppm::g_count[kernel];
    *total_ms = ppm::g_ms[kernel];
    return PPMPM_OK;
}

}  // extern "C"
