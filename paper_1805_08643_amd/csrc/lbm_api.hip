// Host runtime and C ABI (include/mrt_lbm.h) of the MI355X lattice
// Boltzmann library.  The library owns host-side state only; all device
// memory comes from the caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mrt_lbm.h"
#include "lbm_kernels.hpp"

using namespace lbm;

// Scratch of the allocation-free step (lbm_step_noalloc): one copy per GPU,
// resident from the library's load until the process ends.  In host code the
// name is only a stand-in for the symbol: its device address comes from
// hipGetSymbolAddress (scratch_of_current_device below).
static __device__ __align__(256) unsigned char scratch[LBM_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

lbm_status fail(lbm_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(LBM_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                        __FILE__, __LINE__);                                                   \
    } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

size_t elem_bytes(int storage) { return storage == LBM_STORE_F64 ? 8 : (storage == LBM_STORE_F32 ? 4 : 2); }
// Storage elements per node of a population array (19 directions, plus the
// reference plane of F16N).
// Bytes of one population buffer: the planes of N nodes, then the tail
// (F16N: the rounding seed).
size_t pop_bytes(int storage, size_t N) {
    return ((size_t)planes_of(storage) * N + (size_t)tail_elems(storage)) * elem_bytes(storage);
}
size_t real_bytes(int storage) { return storage == LBM_STORE_F64 ? 8 : 4; }

bool rate_ok(double s) { return std::isfinite(s) && s > 0.0 && s < 2.0; }

lbm_status validate(const lbm_params *p) {
    if (!p) return fail(LBM_ERR_INVALID_ARG, "params is NULL");
    if (p->nx < 1 || p->ny < 1 || p->nz < 1)
        return fail(LBM_ERR_INVALID_ARG, "lattice size %d x %d x %d must be positive", p->nx, p->ny, p->nz);
    // In 128-bit integers: three positive 32-bit factors cannot overflow.
    if ((__int128)p->nx * p->ny * p->nz * 19 >= ((__int128)1 << 40))
        return fail(LBM_ERR_INVALID_ARG, "lattice too large");
    if (p->wall_z != 0 && p->wall_z != 1) return fail(LBM_ERR_INVALID_ARG, "wall_z must be 0 or 1");
    if (p->wall_z && p->nz < 2) return fail(LBM_ERR_INVALID_ARG, "walls need nz >= 2");
    if (p->op != LBM_OP_NONORTH && p->op != LBM_OP_ORTH) return fail(LBM_ERR_INVALID_ARG, "unknown op %d", p->op);
    if (p->storage < LBM_STORE_F64 || p->storage > LBM_STORE_F16N)
        return fail(LBM_ERR_INVALID_ARG, "unknown storage %d", p->storage);
    if (p->storage == LBM_STORE_F16N && (p->nx % 4 || p->wall_x || p->wall_y))
        return fail(LBM_ERR_UNSUPPORTED, "F16N storage runs the split step only: nx must be a multiple of 4 (got "
                    "%d) and walls only on z", p->nx);
    if (p->psi_form != LBM_PSI_SQRT_CS && p->psi_form != LBM_PSI_EXP)
        return fail(LBM_ERR_INVALID_ARG, "unknown psi_form %d", p->psi_form);
    if (p->f16_exp < -24 || p->f16_exp > 24) return fail(LBM_ERR_INVALID_ARG, "f16_exp %d outside [-24, 24]", p->f16_exp);
    const double rates[6] = {p->s_e, p->s_nu, p->s_q, p->s_pi, p->s_eps, p->s_m};
    const char *names[6] = {"s_e", "s_nu", "s_q", "s_pi", "s_eps", "s_m"};
    for (int k = 0; k < 6; ++k)
        if (!rate_ok(rates[k])) return fail(LBM_ERR_INVALID_ARG, "%s = %g outside (0, 2)", names[k], rates[k]);
    if (!std::isfinite(p->G)) return fail(LBM_ERR_INVALID_ARG, "G not finite");
    if (p->psi_form == LBM_PSI_SQRT_CS) {
        if (!(p->G < 0.0))
            return fail(LBM_ERR_INVALID_ARG, "square-root pseudopotential needs G < 0 (got %g)", p->G);
        if (!(p->eos_a > 0 && p->eos_b > 0 && p->eos_R > 0 && p->T_over_Tc > 0) || !std::isfinite(p->T_over_Tc))
            return fail(LBM_ERR_INVALID_ARG, "EOS constants a, b, R, T/Tc must be positive");
    } else {
        if (!std::isfinite(p->psi0) || !std::isfinite(p->rho0))
            return fail(LBM_ERR_INVALID_ARG, "psi0, rho0 must be finite");
    }
    if (!std::isfinite(p->sigma)) return fail(LBM_ERR_INVALID_ARG, "sigma not finite");
    if ((p->wall_x != 0 && p->wall_x != 1) || (p->wall_y != 0 && p->wall_y != 1))
        return fail(LBM_ERR_INVALID_ARG, "wall_x and wall_y must be 0 or 1");
    const bool lid = p->lid_u[0] != 0.0 || p->lid_u[1] != 0.0 || p->lid_u[2] != 0.0;
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(p->lid_u[d])) return fail(LBM_ERR_INVALID_ARG, "lid_u not finite");
    if (lid && !p->wall_y) return fail(LBM_ERR_INVALID_ARG, "a moving lid needs wall_y = 1");
    if (lid && p->lid_u[1] != 0.0) return fail(LBM_ERR_INVALID_ARG, "lid_u must be tangential (lid_u[1] = 0)");
    if (lid && !(std::isfinite(p->lid_rho) && p->lid_rho > 0.0))
        return fail(LBM_ERR_INVALID_ARG, "lid_rho must be positive");
    if ((p->wall_x || p->wall_y) && !(p->psi_form == LBM_PSI_EXP && p->G == 0.0))
        return fail(LBM_ERR_UNSUPPORTED, "walls on x or y are implemented for single-phase runs (exponential "
                                         "psi with G = 0)");
    if (!(std::isfinite(p->nu_ratio) && p->nu_ratio >= 0.0))
        return fail(LBM_ERR_INVALID_ARG, "nu_ratio = %g must be finite and >= 0", p->nu_ratio);
    if (p->nu_ratio > 0.0 && p->nu_ratio != 1.0 &&
        !(std::isfinite(p->visc_rho_L) && p->visc_rho_V >= 0.0 && p->visc_rho_L > p->visc_rho_V))
        return fail(LBM_ERR_INVALID_ARG, "variable viscosity needs 0 <= visc_rho_V < visc_rho_L (got %g, %g)",
                    p->visc_rho_V, p->visc_rho_L);
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(p->gravity[d])) return fail(LBM_ERR_INVALID_ARG, "gravity not finite");
    if (p->diag_every < 0) return fail(LBM_ERR_INVALID_ARG, "diag_every must be >= 0");
    if ((p->orth_meq != 0 && p->orth_meq != 1) || (p->orth_sigma != 0 && p->orth_sigma != 1))
        return fail(LBM_ERR_INVALID_ARG, "orth_meq and orth_sigma must be 0 or 1");
    if (!(p->theta_wall_deg > 0.0 && p->theta_wall_deg < 180.0))
        return fail(LBM_ERR_INVALID_ARG, "theta_wall_deg must be in (0, 180)");
    if (!std::isfinite(p->rho_ref) || !std::isfinite(p->ghost_rho_min))
        return fail(LBM_ERR_INVALID_ARG, "rho_ref / ghost_rho_min not finite");
    // Kernels address five direction planes through one buffer descriptor
    // with 32-bit offsets.
    const unsigned long long plane_bytes = (unsigned long long)p->nx * p->ny * p->nz *
                                           (p->storage == LBM_STORE_F64 ? 8 : (p->storage == LBM_STORE_F32 ? 4 : 2));
    if (5 * plane_bytes >= (1ULL << 32))
        return fail(LBM_ERR_UNSUPPORTED,
                    "lattice too large: five population planes take %llu bytes (limit 4 GiB)", 5 * plane_bytes);
    return LBM_OK;
}

PhysD make_phys(const lbm_params &p) {
    PhysD d{};
    d.G = p.G;
    d.a = p.eos_a;
    d.b = p.eos_b;
    // T = (T/Tc) T_c with T_c = 0.37733 a / (b R), text after Eq. (58)
    d.RT = p.eos_R * p.T_over_Tc * 0.37733 * p.eos_a / (p.eos_b * p.eos_R);
    d.psi0 = p.psi0;
    d.rho0 = p.rho0;
    d.s_e = p.s_e;
    d.s_nu = p.s_nu;
    d.s_q = p.s_q;
    d.s_pi = p.s_pi;
    d.s_eps = p.s_eps;
    d.s_m = p.s_m;
    d.sigma = p.sigma;
    for (int k = 0; k < 3; ++k) d.g[k] = p.gravity[k];
    d.tan_wall = std::tan((90.0 - p.theta_wall_deg) * M_PI / 180.0);
    d.ghost_rho_min = p.ghost_rho_min;
    d.rho_ref = p.storage == LBM_STORE_F16S ? p.rho_ref : 0.0;
    d.h_exp = (p.storage == LBM_STORE_F16S || p.storage == LBM_STORE_F16N) ? p.f16_exp : 0;
    d.psi_form = p.psi_form;
    // Density-dependent viscosity: nu = nuV + t dnu, t = (rho - vrhoV) vinv in [0, 1]
    for (int k = 0; k < 3; ++k) d.lid6[k] = 6.0 * p.lid_rho * p.lid_u[k];
    // Orthogonal operator's free equilibrium parameters and Eq. (16) rows.
    d.w_eps = p.orth_meq ? 0.0 : 3.0;
    d.w_epsj = p.orth_meq ? -475.0 / 63.0 : -5.5;
    d.w_xx = p.orth_meq ? 0.0 : -0.5;
    d.sig_eps = p.orth_sigma ? 1.0 : 0.0;
    d.visc = p.nu_ratio > 0.0 && p.nu_ratio != 1.0;
    if (d.visc) {
        const double nuL = (1.0 / p.s_nu - 0.5) / 3.0;
        d.nuV = p.nu_ratio * nuL;
        d.dnu = nuL - d.nuV;
        d.vrhoV = p.visc_rho_V;
        d.vinv = 1.0 / (p.visc_rho_L - p.visc_rho_V);
    }
    return d;
}

struct Layout {
    size_t A, B, psi, rho_w, gpsi, partial, dout, total;
};

Layout layout_of(const lbm_params &p) {
    const size_t N = (size_t)p.nx * p.ny * p.nz;
    const size_t plane = (size_t)p.nx * p.ny;
    const size_t pops = align_up(pop_bytes(p.storage, N));
    Layout L{};
    size_t off = 0;
    L.A = off;
    off += pops;
    L.B = off;
    off += pops;
    L.psi = off;
    off += align_up(N * real_bytes(p.storage));
    L.rho_w = off;
    off += align_up(4 * plane * real_bytes(p.storage));
    L.gpsi = off;
    off += align_up(2 * plane * real_bytes(p.storage));
    L.partial = off;
    off += align_up(sizeof(double) * DIAG_BLOCKS * NDIAG);
    L.dout = off;
    off += align_up(sizeof(double) * NDIAG);
    L.total = off;
    return L;
}

// Threads of a step block: one per npt interior columns (npt = 1, 2 or 4
// x-adjacent nodes per thread), and at least one per halo-ring node.
int block_threads(int tx, int ty, int npt = 1) {
    const int nh = 2 * (tx + 2) + 2 * ty;
    const int n = std::max((tx / npt) * ty, nh);
    return (n + 63) / 64 * 64;
}

// Nodes per thread of a step mode (the split mode moves 8 bytes per access:
// four F16S or two FP32 nodes).
int npt_of(int mode, int storage) {
    if (mode == LBM_STEP_SPLIT) return (storage == ST_F16S || storage == ST_F16N) ? 4 : 2;
    return mode == LBM_STEP_QUADS ? 4 : (mode == LBM_STEP_PAIRS ? 2 : 1);
}

constexpr size_t kMaxStepLds = 65536;

// The split kernel's LDS holds tiles of up to SPLIT_TX x SPLIT_TY nodes,
// SPLIT_ROLE quads per role.
// Rounds of 256 threads that a split tile's halo ring may take: the pullers'
// and the colliders' (one for F16S groups of four, two for FP32 pairs).
int split_rounds(int npt) { return npt == 4 ? 2 : 3; }

// Slots of the split step's psi ring: (tx + 2)(ty + 2) of a tile at most
// (F16N's LDS also holds a ring of reference densities, so its tiles are smaller).
int split_sp(int storage) { return storage == ST_F16N ? SPLIT_SP_N : SPLIT_SP; }

lbm_status check_split_tile(const lbm_tile &t, int npt, int storage) {
    // The halo ring, 2 (tx + 2) + 2 ty nodes, takes at most split_rounds(npt)
    // rounds of 256 threads (pullers, then colliders once for F16S, twice for FP32).
    const int ring_max = split_rounds(npt) * SPLIT_ROLE / 2 - 2;
    const int sp = split_sp(storage);
    if (t.tx < npt || t.ty < 1 || t.cz < 1 || t.tx % npt || t.tx > SPLIT_TX || (t.tx / npt) * t.ty > SPLIT_ROLE ||
        t.tx * t.ty > SPLIT_NODES || (t.tx + 2) * (t.ty + 2) > sp || t.tx + t.ty > ring_max)
        return fail(LBM_ERR_INVALID_ARG, "split mode needs a tile width that is a multiple of %d and at most %d, at "
                    "most %d groups of %d nodes, %d nodes, (tx + 2)(ty + 2) <= %d and tx + ty <= %d; got %d x %d x %d",
                    npt, SPLIT_TX, SPLIT_ROLE, npt, SPLIT_NODES, sp, ring_max, t.tx, t.ty, t.cz);
    return LBM_OK;
}

// Last-level cache (Infinity Cache) of the MI355X: population arrays larger
// than this stream through it, and the split step stores them non-temporally.
constexpr size_t kLlcBytes = 256ull << 20;
bool stream_stores(int policy, size_t pop_bytes) {
    return policy == LBM_STORE_STREAM || (policy == LBM_STORE_AUTO && pop_bytes > kLlcBytes);
}

// Whether a split tile's halo ring has more nodes than the pulling threads.
bool split_ring2(int tx, int ty) { return 2 * (tx + 2) + 2 * ty > SPLIT_ROLE; }

// Most rows a split tile of width tx can have.
int split_rows(int tx, int npt, int storage) {
    return std::max(1, std::min({SPLIT_ROLE / (tx / npt), SPLIT_NODES / tx, split_sp(storage) / (tx + 2) - 2,
                                 split_rounds(npt) * SPLIT_ROLE / 2 - 2 - tx}));
}

lbm_status check_tile(const lbm_tile &t, int storage, int npt = 1) {
    if (t.tx < 1 || t.ty < 1 || t.cz < 1) return fail(LBM_ERR_INVALID_ARG, "tile dims must be positive");
    if (t.tx > 1024 || t.ty > 1024) return fail(LBM_ERR_INVALID_ARG, "tile dims must be <= 1024");
    if (t.tx % npt)
        return fail(LBM_ERR_INVALID_ARG, "%d nodes per thread need a tile width that is a multiple of %d, got %d",
                    npt, npt, t.tx);
    if ((t.tx / npt) * t.ty > STEP_MAX_THREADS || block_threads(t.tx, t.ty, npt) > STEP_MAX_THREADS)
        return fail(LBM_ERR_INVALID_ARG, "tile %d x %d needs more than %d threads", t.tx, t.ty, STEP_MAX_THREADS);
    if (4 * (size_t)(t.ty + 2) * (t.tx + 2) * real_bytes(storage) > kMaxStepLds)
        return fail(LBM_ERR_INVALID_ARG, "tile %d x %d needs more than %zu bytes of LDS", t.tx, t.ty, kMaxStepLds);
    return LBM_OK;
}

void fill_grid(GridDesc &g, const lbm_params &p, const lbm_tile &t) {
    g.nx = p.nx;
    g.ny = p.ny;
    g.nz = p.nz;
    g.wall = p.wall_z;
    g.wall_x = p.wall_x;
    g.wall_y = p.wall_y;
    g.N = (long long)p.nx * p.ny * p.nz;
    g.tx = t.tx;
    g.ty = t.ty;
    g.cz = std::min(t.cz, p.nz);
    g.ntx = (p.nx + t.tx - 1) / t.tx;
    g.nty = (p.ny + t.ty - 1) / t.ty;
    g.nzc = (p.nz + g.cz - 1) / g.cz;
    g.ntiles = g.ntx * g.nty * g.nzc;
    g.per_xcd = (g.ntiles + 7) / 8;
}

lbm_tile default_tile(int nx, int ny, int nz) {
    lbm_tile t{};
    // x extent: whole row when short, otherwise the candidate of 64 or 32
    // that wastes fewest columns.
    if (nx <= 64) {
        t.tx = nx;
    } else {
        const int w64 = (nx + 63) / 64 * 64 - nx, w32 = (nx + 31) / 32 * 32 - nx;
        t.tx = w64 <= w32 ? 64 : 32;
    }
    t.ty = std::max(1, std::min(ny, STEP_MAX_THREADS / t.tx));
    while (t.ty > 1 && block_threads(t.tx, t.ty) > STEP_MAX_THREADS) --t.ty;
    while (block_threads(t.tx, t.ty) > STEP_MAX_THREADS && t.tx > 1) t.tx /= 2;
    const int ncol = ((nx + t.tx - 1) / t.tx) * ((ny + t.ty - 1) / t.ty);
    const int want = 2048;  // ~8 blocks per CU
    int nzc = std::max(1, (want + ncol - 1) / ncol);
    int cz = std::max(1, (nz + nzc - 1) / nzc);
    cz = std::max(cz, std::min(nz, 8));
    t.cz = cz;
    return t;
}

// Default tile with npt = 2 or 4 nodes per thread: rows of up to 128
// columns, up to 512 interior threads, and z runs long enough that there are
// about as many tiles as compute units (measured fastest at 256^3: 128 x 8 x
// 64 with pairs).
lbm_tile wide_tile(int nx, int ny, int nz, int npt) {
    lbm_tile t{};
    t.tx = std::min(nx, 128);
    t.tx = (t.tx + npt - 1) / npt * npt;
    t.ty = std::max(1, std::min(ny, STEP_MAX_THREADS / std::max(1, t.tx / npt)));
    while (t.ty > 1 && block_threads(t.tx, t.ty, npt) > STEP_MAX_THREADS) --t.ty;
    const int ncol = ((nx + t.tx - 1) / t.tx) * ((ny + t.ty - 1) / t.ty);
    const int nzc = std::max(1, (256 + ncol - 1) / ncol);
    t.cz = std::max(std::min(nz, 8), (nz + nzc - 1) / nzc);
    return t;
}

bool box_walls(const lbm_params &p) { return p.wall_x || p.wall_y; }
bool pairs_apply(const lbm_params &p) {
    return (p.storage == ST_F32 || p.storage == ST_F16S) && p.nx % 2 == 0 && !box_walls(p);
}
bool quads_apply(const lbm_params &p) { return p.storage == ST_F16S && p.nx % 4 == 0 && !box_walls(p); }
bool split_apply(const lbm_params &p) {
    return !box_walls(p) && (((p.storage == ST_F16S || p.storage == ST_F16N) && p.nx % 4 == 0) ||
                             (p.storage == ST_F32 && p.nx % 2 == 0));
}

// Default tile of the split mode: rows of up to 128 nodes, up to
// SPLIT_ROLE groups, z runs for about as many tiles as compute units.
constexpr int SPLIT_TX_DEFAULT = 128;
lbm_tile split_tile(int nx, int ny, int nz, int npt, int storage) {
    lbm_tile t{};
    t.tx = std::min(SPLIT_TX_DEFAULT, (nx + npt - 1) / npt * npt);
    t.ty = std::max(1, std::min({ny, SPLIT_TY, split_rows(t.tx, npt, storage)}));
    const int ncol = ((nx + t.tx - 1) / t.tx) * ((ny + t.ty - 1) / t.ty);
    const int nzc = std::max(1, (256 + ncol - 1) / ncol);
    t.cz = std::max(std::min(nz, 8), (nz + nzc - 1) / nzc);
    return t;
}

}  // namespace

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct lbm_ctx {
    lbm_params p{};
    PhysD pd{};
    GridDesc g{};
    lbm_tile tile{};
    Layout L{};
    hipStream_t stream = nullptr;
    unsigned char *ws = nullptr;
    int cur = 0;  // 0: state in A; 1: state in B
    int64_t steps = 0;
    bool timing = false;
    std::vector<hipEvent_t> ev;  // start/stop pairs
    size_t nev = 0;              // pairs recorded since last read
    int mode = LBM_STEP_FUSED;
    int slab = 32;
    bool write_check = false;
    int store_policy = LBM_STORE_AUTO;
    int graph_steps = 0;                         // 0: plain launches
    hipStream_t cap = nullptr;                   // capture stream of the graphs
    hipGraphExec_t graphs[2] = {nullptr, nullptr};  // k steps from buffer parity 0 / 1

    // Wall-plane densities and ghost psi (Eq. (57)) in a buffer of their own
    // instead of the workspace: the allocation-free step (lbm_step_noalloc).
    unsigned char *wall_scratch = nullptr;

    void *state() const { return ws + (cur ? L.B : L.A); }
    void *other() const { return ws + (cur ? L.A : L.B); }
    void *psi() const { return ws + L.psi; }
    void *rho_w() const { return wall_scratch ? wall_scratch : ws + L.rho_w; }
    void *gpsi() const { return wall_scratch ? wall_scratch + (L.gpsi - L.rho_w) : ws + L.gpsi; }
    double *partial() const { return reinterpret_cast<double *>(ws + L.partial); }
    double *dout() const { return reinterpret_cast<double *>(ws + L.dout); }
};

namespace {

unsigned grid1d(long long n, int threads, long long cap = 65536) {
    long long b = (n + threads - 1) / threads;
    return (unsigned)std::max(1LL, std::min(b, cap));
}

// Template dispatch over storage, operator and wall mode.
template <class F> lbm_status dispatch(const lbm_ctx *c, F &&fn) {
    const int S = c->p.storage, O = c->p.op;
    const bool W = c->p.wall_z != 0;
#define LBM_CASE(s, o, w) \
    if (S == s && O == o && W == w) return fn(std::integral_constant<int, s>{}, std::integral_constant<int, o>{}, std::integral_constant<bool, w>{});
    LBM_CASE(ST_F64, OP_NONORTH, false)
    LBM_CASE(ST_F64, OP_NONORTH, true)
    LBM_CASE(ST_F64, OP_ORTH, false)
    LBM_CASE(ST_F64, OP_ORTH, true)
    LBM_CASE(ST_F32, OP_NONORTH, false)
    LBM_CASE(ST_F32, OP_NONORTH, true)
    LBM_CASE(ST_F32, OP_ORTH, false)
    LBM_CASE(ST_F32, OP_ORTH, true)
    LBM_CASE(ST_F16S, OP_NONORTH, false)
    LBM_CASE(ST_F16S, OP_NONORTH, true)
    LBM_CASE(ST_F16S, OP_ORTH, false)
    LBM_CASE(ST_F16S, OP_ORTH, true)
    LBM_CASE(ST_F16N, OP_NONORTH, false)
    LBM_CASE(ST_F16N, OP_NONORTH, true)
    LBM_CASE(ST_F16N, OP_ORTH, false)
    LBM_CASE(ST_F16N, OP_ORTH, true)
#undef LBM_CASE
    return fail(LBM_ERR_UNSUPPORTED, "no kernel for storage %d op %d wall %d", S, O, (int)W);
}

lbm_status launch_walls(lbm_ctx *c, const void *src) {
    return dispatch(c, [&](auto S, auto, auto W) -> lbm_status {
        using T = typename Storage<S.value>::T;
        using R = typename Storage<S.value>::R;
        if (!W.value) return LBM_OK;
        const long long plane = (long long)c->p.nx * c->p.ny;
        hipLaunchKernelGGL(k_wall_rho<S.value>, dim3(grid1d(4 * plane, 256, 1LL << 30)), dim3(256), 0, c->stream,
                           (const T *)src, (R *)c->rho_w(), c->g, c->pd);
        hipLaunchKernelGGL(k_ghost_psi<R>, dim3(grid1d(2 * plane, 256, 1LL << 30)), dim3(256), 0, c->stream,
                           (const R *)c->rho_w(), (R *)c->gpsi(), c->g, c->pd);
        HIP_TRY(hipGetLastError());
        return LBM_OK;
    });
}

size_t step_smem(const lbm_ctx *c, const GridDesc &g) {
    return 4 * (size_t)(g.ty + 2) * (g.tx + 2) * real_bytes(c->p.storage);
}

lbm_status launch_step(lbm_ctx *c, const GridDesc &g, const void *src, void *dst, int npt) {
    return dispatch(c, [&](auto S, auto O, auto W) -> lbm_status {
        using T = typename Storage<S.value>::T;
        using R = typename Storage<S.value>::R;
        if constexpr (S.value == ST_F16N) {
            // validate() admits F16N only where the split step runs.
            if (c->mode != LBM_STEP_SPLIT) return fail(LBM_ERR_UNSUPPORTED, "F16N storage runs the split step only");
        } else if (box_walls(c->p)) {  // single phase with walls on x or y: own kernel
            hipLaunchKernelGGL((k_single<S.value, O.value>), dim3(grid1d(g.N, 256, 1LL << 30)), dim3(256), 0,
                               c->stream, (const T *)src, (T *)dst, g, c->pd);
            HIP_TRY(hipGetLastError());
            return LBM_OK;
        }
        const unsigned grid = 8u * (unsigned)g.per_xcd;
        const int threads = block_threads(g.tx, g.ty, npt);
        if (c->mode != LBM_STEP_SPLIT && threads > STEP_MAX_THREADS)
            return fail(LBM_ERR_INVALID_ARG, "tile %d x %d at %d node(s) per thread needs %d threads, more than %d",
                        g.tx, g.ty, npt, threads, STEP_MAX_THREADS);
        if (c->mode == LBM_STEP_SPLIT) {
            if constexpr (S.value != ST_F64) {
                lbm_tile t{g.tx, g.ty, g.cz, 0};
                if (g.nx % npt) return fail(LBM_ERR_INVALID_ARG, "split mode needs nx a multiple of %d", npt);
                if (lbm_status e = check_split_tile(t, npt, S.value)) return e;
                const bool r2 = split_ring2(g.tx, g.ty);
                const bool nt = stream_stores(c->store_policy, 2 * (c->L.B - c->L.A));
#define LBM_SPLIT_LAUNCH(R2, NT)                                                                              \
    hipLaunchKernelGGL((k_step_split<S.value, O.value, W.value, R2, NT>), dim3(grid), dim3(2 * SPLIT_ROLE), 0, \
                       c->stream, (const T *)src, (T *)dst, (const R *)c->gpsi(), g, c->pd)
                if constexpr (S.value == ST_F16N) {
                    // The pullers take the whole halo ring, in a second round
                    // where it has more nodes than pullers: with the colliders
                    // sharing it (RING2) the F16N step measured 43% slower
                    // (0.474 against 0.332 ms at 256^3, 128 x 8 x 64 tiles).
                    if (nt) LBM_SPLIT_LAUNCH(false, true);
                    else LBM_SPLIT_LAUNCH(false, false);
                } else {
                    if (r2 && nt) LBM_SPLIT_LAUNCH(true, true);
                    else if (r2) LBM_SPLIT_LAUNCH(true, false);
                    else if (nt) LBM_SPLIT_LAUNCH(false, true);
                    else LBM_SPLIT_LAUNCH(false, false);
                }
#undef LBM_SPLIT_LAUNCH
                HIP_TRY(hipGetLastError());
                return LBM_OK;
            } else {
                return fail(LBM_ERR_UNSUPPORTED, "split mode needs FP32 or F16S storage");
            }
        }
        if constexpr (S.value == ST_F16N) {
            return LBM_OK;  // not reached: the split step returned above
        } else {
        if (npt == 4) {
            if constexpr (S.value == ST_F16S) {
                // nx and tx multiples of 4: checked by lbm_set_step_mode / lbm_set_tile
                if (g.nx % 4 || g.tx % 4) return fail(LBM_ERR_INVALID_ARG, "quad mode needs nx and tile width % 4 == 0");
                hipLaunchKernelGGL((k_step4<O.value, W.value>), dim3(grid), dim3(threads), step_smem(c, g), c->stream,
                                   (const T *)src, (T *)dst, (const R *)c->gpsi(), g, c->pd);
                HIP_TRY(hipGetLastError());
                return LBM_OK;
            } else {
                return fail(LBM_ERR_UNSUPPORTED, "quad mode needs F16S storage");
            }
        }
        const bool pairs = npt == 2;
        if constexpr (S.value != ST_F64) {
            if (pairs) {
                // even nx and tx: checked by lbm_set_step_mode / lbm_set_tile
                if (g.nx % 2 || g.tx % 2) return fail(LBM_ERR_INVALID_ARG, "pair mode needs even nx and tile width");
                hipLaunchKernelGGL((k_step2<S.value, O.value, W.value>), dim3(grid), dim3(threads), step_smem(c, g),
                                   c->stream, (const T *)src, (T *)dst, (const R *)c->gpsi(), g, c->pd);
                HIP_TRY(hipGetLastError());
                return LBM_OK;
            }
        } else if (pairs) {
            return fail(LBM_ERR_UNSUPPORTED, "pair mode needs FP32 or F16S storage");
        }
        hipLaunchKernelGGL((k_step<S.value, O.value, W.value>), dim3(grid), dim3(threads), step_smem(c, g),
                           c->stream, (const T *)src, (T *)dst, (const R *)c->gpsi(), g, c->pd);
        HIP_TRY(hipGetLastError());
        return LBM_OK;
        }
    });
}

lbm_status launch_slabs(lbm_ctx *c, const void *src, void *dst) {
    return dispatch(c, [&](auto S, auto O, auto W) -> lbm_status {
        using T = typename Storage<S.value>::T;
        using R = typename Storage<S.value>::R;
        if constexpr (S.value == ST_F16N) {
            return fail(LBM_ERR_UNSUPPORTED, "F16N storage runs the split step only");
        } else {
        const int nz = c->p.nz;
        const long long plane = (long long)c->p.nx * c->p.ny;
        auto psi_pass = [&](int za, int zb) {
            if (zb <= za) return;
            hipLaunchKernelGGL((k_psi_planes<S.value, W.value>), dim3(grid1d(plane * (zb - za), 256)), dim3(256), 0,
                               c->stream, (const T *)src, (R *)c->psi(), c->g, c->pd, za, zb);
        };
        // psi of the planes below the first slab: plane 0, and plane nz-1 for
        // the periodic wrap (walls use the ghost layer instead).
        psi_pass(0, 1);
        if (!W.value && nz > 1) psi_pass(nz - 1, nz);
        for (int z0 = 0; z0 < nz; z0 += c->slab) {
            const int z1 = std::min(nz, z0 + c->slab);
            psi_pass(z0 + 1, std::min(z1 + 1, nz));
            hipLaunchKernelGGL((k_collide_planes<S.value, O.value, W.value>), dim3(grid1d(plane * (z1 - z0), 256)),
                               dim3(256), 0, c->stream, (const T *)src, (T *)dst, (const R *)c->psi(),
                               (const R *)c->gpsi(), c->g, c->pd, z0, z1);
        }
        HIP_TRY(hipGetLastError());
        return LBM_OK;
        }
    });
}

lbm_status timed_event(lbm_ctx *c, size_t k) {
    while (c->ev.size() <= k) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        c->ev.push_back(e);
    }
    HIP_TRY(hipEventRecord(c->ev[k], c->stream));
    return LBM_OK;
}

// All-ones bits over n 16-bit words: NaN in every storage format.
__global__ void __launch_bounds__(256) k_fill_ones(uint16_t *p, long long n) {
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) p[i] = 0xFFFFu;
}

lbm_status one_step(lbm_ctx *c) {
    lbm_status s = launch_walls(c, c->state());
    if (s) return s;
    if (c->write_check) {
        const long long words = (long long)(pop_bytes(c->p.storage, (size_t)c->g.N) / 2);
        hipLaunchKernelGGL(k_fill_ones, dim3(grid1d(words, 256)), dim3(256), 0, c->stream,
                           (uint16_t *)c->other(), words);
        HIP_TRY(hipGetLastError());
    }
    if (c->timing) {
        if ((s = timed_event(c, 2 * c->nev))) return s;
    }
    if (c->mode == LBM_STEP_SLABS && !box_walls(c->p)) {
        if ((s = launch_slabs(c, c->state(), c->other()))) return s;
    } else if ((s = launch_step(c, c->g, c->state(), c->other(), npt_of(c->mode, c->p.storage)))) {
        return s;
    }
    if (c->timing) {
        if ((s = timed_event(c, 2 * c->nev + 1))) return s;
        ++c->nev;
    }
    c->cur ^= 1;
    ++c->steps;
    return LBM_OK;
}

// Default step of a new context: the split step where it applies (the
// fastest on every workload measured), else two nodes per thread, else one.
void default_mode(lbm_ctx *c) {
    const lbm_params &p = c->p;
    if (split_apply(p)) {
        c->mode = LBM_STEP_SPLIT;
        c->tile = split_tile(p.nx, p.ny, p.nz, npt_of(LBM_STEP_SPLIT, p.storage), p.storage);
    } else if (pairs_apply(p)) {
        c->mode = LBM_STEP_PAIRS;
        c->tile = wide_tile(p.nx, p.ny, p.nz, 2);
    } else {
        c->mode = LBM_STEP_FUSED;
        c->tile = default_tile(p.nx, p.ny, p.nz);
    }
    fill_grid(c->g, p, c->tile);
}

// Device address of the allocation-free step's scratch array on the current
// device: looked up once per device with hipGetSymbolAddress (with that device
// current) and kept; host code passes only this pointer to kernels.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

lbm_status scratch_of_current_device(unsigned char **out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LBM_ERR_UNSUPPORTED, "device index %d >= %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(LBM_ERR_HIP, "no device address for the scratch array on device %d", dev);
        g_scratch_ptr[dev] = static_cast<unsigned char *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}

void drop_graphs(lbm_ctx *c) {
    for (hipGraphExec_t &g : c->graphs) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

// k steps of the current parity from a captured graph (captured on first use
// on the context's capture stream; the context's counters are advanced here,
// not by the capture).
lbm_status graph_steps(lbm_ctx *c, int k) {
    hipGraphExec_t &ex = c->graphs[c->cur];
    if (!ex) {
        if (!c->cap) HIP_TRY(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
        const hipStream_t user = c->stream;
        const int cur0 = c->cur;
        const int64_t steps0 = c->steps;
        HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
        c->stream = c->cap;
        lbm_status s = LBM_OK;
        for (int j = 0; j < k && s == LBM_OK; ++j) s = one_step(c);
        c->stream = user;
        c->cur = cur0;
        c->steps = steps0;
        hipGraph_t graph;
        hipError_t e = hipStreamEndCapture(c->cap, &graph);
        if (s) {
            if (e == hipSuccess) (void)hipGraphDestroy(graph);
            return s;
        }
        if (e != hipSuccess) return fail(LBM_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            ex = nullptr;
            return fail(LBM_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
    }
    HIP_TRY(hipGraphLaunch(ex, c->stream));
    c->cur ^= (k & 1);
    c->steps += k;
    return LBM_OK;
}

lbm_status compute_psi_full(lbm_ctx *c) {
    lbm_status s = launch_walls(c, c->state());
    if (s) return s;
    return dispatch(c, [&](auto S, auto, auto W) -> lbm_status {
        using T = typename Storage<S.value>::T;
        using R = typename Storage<S.value>::R;
        hipLaunchKernelGGL((k_psi_full<S.value, W.value>), dim3(grid1d(c->g.N, 256)), dim3(256), 0, c->stream,
                           (const T *)c->state(), (R *)c->psi(), c->g, c->pd);
        HIP_TRY(hipGetLastError());
        return LBM_OK;
    });
}

}  // namespace

extern "C" {

void lbm_params_default(lbm_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->nx = p->ny = p->nz = 32;
    p->wall_z = 0;
    p->op = LBM_OP_NONORTH;
    p->storage = LBM_STORE_F32;
    p->psi_form = LBM_PSI_SQRT_CS;
    p->rho_ref = 0.0;
    p->s_e = p->s_nu = p->s_q = p->s_pi = p->s_eps = p->s_m = 1.0;
    p->G = -1.0;
    p->eos_a = 0.5;
    p->eos_b = 4.0;
    p->eos_R = 1.0;
    p->T_over_Tc = 0.8;
    p->psi0 = 1.0;
    p->rho0 = 1.0;
    p->sigma = 0.0;
    p->theta_wall_deg = 90.0;
    p->ghost_rho_min = 0.0;
}

lbm_status lbm_workspace_bytes(const lbm_params *p, size_t *bytes) {
    lbm_status s = validate(p);
    if (s) return s;
    if (!bytes) return fail(LBM_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = layout_of(*p).total;
    return LBM_OK;
}

lbm_status lbm_create(const lbm_params *p, void *dev_ws, size_t ws_bytes, void *hip_stream, lbm_ctx **out) {
    lbm_status s = validate(p);
    if (s) return s;
    if (!out) return fail(LBM_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!dev_ws) return fail(LBM_ERR_INVALID_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(dev_ws) % kAlign)
        return fail(LBM_ERR_INVALID_ARG, "workspace must be %zu-byte aligned", kAlign);
    Layout L = layout_of(*p);
    if (ws_bytes < L.total)
        return fail(LBM_ERR_BUFFER_TOO_SMALL, "workspace %zu bytes < required %zu", ws_bytes, L.total);
    lbm_ctx *c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(LBM_ERR_INVALID_ARG, "out of host memory");
    c->p = *p;
    c->pd = make_phys(*p);
    c->L = L;
    c->ws = static_cast<unsigned char *>(dev_ws);
    c->stream = static_cast<hipStream_t>(hip_stream);
    default_mode(c);
    *out = c;
    return LBM_OK;
}

lbm_status lbm_destroy(lbm_ctx *c) {
    if (!c) return fail(LBM_ERR_INVALID_ARG, "ctx is NULL");
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    drop_graphs(c);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    delete c;
    return LBM_OK;
}

lbm_status lbm_init_fields(lbm_ctx *c, const double *rho, const double *u) {
    if (!c || !rho || !u) return fail(LBM_ERR_INVALID_ARG, "null argument");
    lbm_status s = dispatch(c, [&](auto S, auto O, auto W) -> lbm_status {
        using T = typename Storage<S.value>::T;
        hipLaunchKernelGGL((k_init_fields<S.value, O.value, W.value>), dim3(grid1d(c->g.N, 256)), dim3(256), 0,
                           c->stream, (T *)c->state(), rho, u, c->g, c->pd);
        HIP_TRY(hipGetLastError());
        return LBM_OK;
    });
    if (s == LBM_OK) c->steps = 0;
    return s;
}

lbm_status lbm_init_droplets(lbm_ctx *c, const lbm_droplet *d, int32_t n, double rho_L, double rho_V, double W) {
    if (!c || !d) return fail(LBM_ERR_INVALID_ARG, "null argument");
    if (n < 1 || n > 8) return fail(LBM_ERR_INVALID_ARG, "droplet count %d outside [1, 8]", n);
    if (!(W > 0) || !(rho_L > 0) || !(rho_V > 0)) return fail(LBM_ERR_INVALID_ARG, "need W, rho_L, rho_V > 0");
    DropletSet D{};
    D.n = n;
    D.rho_L = rho_L;
    D.rho_V = rho_V;
    D.W = W;
    for (int k = 0; k < n; ++k) {
        for (int a = 0; a < 3; ++a) {
            D.c[k][a] = d[k].center[a];
            D.u[k][a] = d[k].u[a];
        }
        D.r0[k] = d[k].r0;
    }
    lbm_status s = dispatch(c, [&](auto S, auto O, auto Wl) -> lbm_status {
        using T = typename Storage<S.value>::T;
        hipLaunchKernelGGL((k_init_droplets<S.value, O.value, Wl.value>), dim3(grid1d(c->g.N, 256)), dim3(256), 0,
                           c->stream, (T *)c->state(), D, c->g, c->pd);
        HIP_TRY(hipGetLastError());
        return LBM_OK;
    });
    if (s == LBM_OK) c->steps = 0;
    return s;
}

lbm_status lbm_step(lbm_ctx *c, int64_t nsteps) {
    if (!c) return fail(LBM_ERR_INVALID_ARG, "ctx is NULL");
    if (nsteps < 0) return fail(LBM_ERR_INVALID_ARG, "nsteps < 0");
    const int64_t K = c->p.diag_every;
    const int G = c->timing ? 0 : c->graph_steps;
    int64_t left = nsteps;
    while (left > 0) {
        // Run up to the next multiple of diag_every (or to the end).
        int64_t chunk = left;
        if (K > 0) chunk = std::min<int64_t>(left, K - c->steps % K);
        for (int64_t done = 0; done < chunk;) {
            lbm_status s;
            if (G > 0 && chunk - done >= G) {
                s = graph_steps(c, G);
                done += G;
            } else {
                s = one_step(c);
                ++done;
            }
            if (s) return s;
        }
        left -= chunk;
        if (K > 0 && c->steps % K == 0) {
            lbm_diag d;
            lbm_status s = lbm_diagnostics(c, nullptr, &d);
            if (s) return s;  // LBM_ERR_NONFINITE names the step
        }
    }
    return LBM_OK;
}

lbm_status lbm_set_graph_steps(lbm_ctx *c, int32_t k) {
    if (!c) return fail(LBM_ERR_INVALID_ARG, "ctx is NULL");
    if (k < 0) return fail(LBM_ERR_INVALID_ARG, "graph steps %d < 0", k);
    if (k != c->graph_steps) drop_graphs(c);
    c->graph_steps = k;
    return LBM_OK;
}

lbm_status lbm_step_noalloc(const lbm_params *p, const void *dev_src, void *dev_dst, void *hip_stream) {
    lbm_status s = validate(p);
    if (s) return s;
    if (!dev_src || !dev_dst) return fail(LBM_ERR_INVALID_ARG, "population buffer is NULL");
    if (dev_src == dev_dst) return fail(LBM_ERR_INVALID_ARG, "source and destination must differ");
    if (reinterpret_cast<uintptr_t>(dev_src) % kAlign || reinterpret_cast<uintptr_t>(dev_dst) % kAlign)
        return fail(LBM_ERR_INVALID_ARG, "population buffers must be %zu-byte aligned", kAlign);
    // Scratch: the wall-plane densities and the ghost psi planes (walls only).
    const Layout L = layout_of(*p);
    const size_t need = p->wall_z ? L.partial - L.rho_w : 0;
    if (need > (size_t)LBM_NOALLOC_SCRATCH_BYTES)
        return fail(LBM_ERR_UNSUPPORTED, "walled lattice %d x %d needs %zu bytes of scratch, more than the %d of "
                    "lbm_step_noalloc", p->nx, p->ny, need, LBM_NOALLOC_SCRATCH_BYTES);
    unsigned char *scr = nullptr;
    if ((s = scratch_of_current_device(&scr))) return s;
    lbm_ctx c;  // on the stack: no host allocation
    c.p = *p;
    c.pd = make_phys(*p);
    c.L = L;
    c.stream = static_cast<hipStream_t>(hip_stream);
    c.wall_scratch = scr;
    default_mode(&c);
    if ((s = launch_walls(&c, dev_src))) return s;
    return launch_step(&c, c.g, dev_src, dev_dst, npt_of(c.mode, p->storage));
}

lbm_status lbm_read_fields(lbm_ctx *c, double *rho, double *u, double *p) {
    if (!c) return fail(LBM_ERR_INVALID_ARG, "ctx is NULL");
    lbm_status s = compute_psi_full(c);
    if (s) return s;
    return dispatch(c, [&](auto S, auto, auto W) -> lbm_status {
        using T = typename Storage<S.value>::T;
        using R = typename Storage<S.value>::R;
        hipLaunchKernelGGL((k_fields<S.value, W.value>), dim3(grid1d(c->g.N, 256)), dim3(256), 0, c->stream,
                           (const T *)c->state(), (const R *)c->psi(), (const R *)c->gpsi(), rho, u, p, c->g, c->pd);
        HIP_TRY(hipGetLastError());
        return LBM_OK;
    });
}

lbm_status lbm_read_populations(lbm_ctx *c, double *f) {
    if (!c || !f) return fail(LBM_ERR_INVALID_ARG, "null argument");
    return dispatch(c, [&](auto S, auto, auto W) -> lbm_status {
        using T = typename Storage<S.value>::T;
        hipLaunchKernelGGL((k_read_pops<S.value, W.value>), dim3(grid1d(c->g.N, 256)), dim3(256), 0, c->stream,
                           (const T *)c->state(), f, c->g, c->pd);
        HIP_TRY(hipGetLastError());
        return LBM_OK;
    });
}

lbm_status lbm_write_populations(lbm_ctx *c, const double *f) {
    if (!c || !f) return fail(LBM_ERR_INVALID_ARG, "null argument");
    return dispatch(c, [&](auto S, auto, auto W) -> lbm_status {
        using T = typename Storage<S.value>::T;
        hipLaunchKernelGGL((k_write_pops<S.value, W.value>), dim3(grid1d(c->g.N, 256)), dim3(256), 0, c->stream,
                           (T *)c->state(), f, c->g, c->pd);
        HIP_TRY(hipGetLastError());
        return LBM_OK;
    });
}

lbm_status lbm_diagnostics(lbm_ctx *c, const lbm_diag_request *req, lbm_diag *out) {
    if (!c || !out) return fail(LBM_ERR_INVALID_ARG, "null argument");
    DiagReq rq{};
    if (req) {
        if (!(req->r_in >= 0 && req->r_out >= 0)) return fail(LBM_ERR_INVALID_ARG, "radii must be >= 0");
        for (int a = 0; a < 3; ++a) rq.c[a] = req->center[a];
        rq.r_in2 = req->r_in * req->r_in;
        rq.r_out2 = req->r_out * req->r_out;
        rq.enabled = 1;
    }
    lbm_status s = compute_psi_full(c);
    if (s) return s;
    const int nblk = (int)std::min<long long>(DIAG_BLOCKS, (c->g.N + DIAG_THREADS - 1) / DIAG_THREADS);
    s = dispatch(c, [&](auto S, auto, auto W) -> lbm_status {
        using T = typename Storage<S.value>::T;
        using R = typename Storage<S.value>::R;
        hipLaunchKernelGGL((k_diag<S.value, W.value>), dim3(nblk), dim3(DIAG_THREADS), 0, c->stream,
                           (const T *)c->state(), (const R *)c->psi(), (const R *)c->gpsi(), c->partial(), c->g,
                           c->pd, rq);
        hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(DIAG_FINAL_THREADS), 0, c->stream,
                           (const double *)c->partial(), nblk, c->dout());
        HIP_TRY(hipGetLastError());
        return LBM_OK;
    });
    if (s) return s;
    double h[NDIAG];
    HIP_TRY(hipMemcpyAsync(h, c->dout(), sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    out->mass = h[0];
    out->momentum[0] = h[1];
    out->momentum[1] = h[2];
    out->momentum[2] = h[3];
    out->max_u = h[4];
    out->p_in = h[5];
    out->p_out = h[6];
    out->rho_in = h[7];
    out->rho_out = h[8];
    out->n_in = h[9];
    out->n_out = h[10];
    out->nonfinite = (int64_t)h[11];
    out->step = c->steps;
    if (out->nonfinite) return fail(LBM_ERR_NONFINITE, "%lld non-finite populations at step %lld",
                                    (long long)out->nonfinite, (long long)c->steps);
    return LBM_OK;
}

lbm_status lbm_state_bytes(const lbm_ctx *c, size_t *bytes) {
    if (!c || !bytes) return fail(LBM_ERR_INVALID_ARG, "null argument");
    *bytes = pop_bytes(c->p.storage, (size_t)c->g.N) + sizeof(int64_t);
    return LBM_OK;
}

lbm_status lbm_save_state(lbm_ctx *c, void *dev_buf, size_t bytes) {
    size_t need = 0;
    lbm_status s = lbm_state_bytes(c, &need);
    if (s) return s;
    if (!dev_buf) return fail(LBM_ERR_INVALID_ARG, "buffer is NULL");
    if (bytes < need) return fail(LBM_ERR_BUFFER_TOO_SMALL, "state buffer %zu < %zu", bytes, need);
    const size_t pb = need - sizeof(int64_t);
    HIP_TRY(hipMemcpyAsync(dev_buf, c->state(), pb, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(static_cast<unsigned char *>(dev_buf) + pb, &c->steps, sizeof(int64_t),
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_load_state(lbm_ctx *c, const void *dev_buf, size_t bytes) {
    size_t need = 0;
    lbm_status s = lbm_state_bytes(c, &need);
    if (s) return s;
    if (!dev_buf) return fail(LBM_ERR_INVALID_ARG, "buffer is NULL");
    if (bytes < need) return fail(LBM_ERR_BUFFER_TOO_SMALL, "state buffer %zu < %zu", bytes, need);
    const size_t pb = need - sizeof(int64_t);
    int64_t st = 0;
    HIP_TRY(hipMemcpyAsync(c->state(), dev_buf, pb, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(&st, static_cast<const unsigned char *>(dev_buf) + pb, sizeof(int64_t),
                           hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->steps = st;
    return LBM_OK;
}

lbm_status lbm_set_tile(lbm_ctx *c, const lbm_tile *t) {
    if (!c || !t) return fail(LBM_ERR_INVALID_ARG, "null argument");
    const int npt = npt_of(c->mode, c->p.storage);
    lbm_status s = c->mode == LBM_STEP_SPLIT ? check_split_tile(*t, npt, c->p.storage)
                                             : check_tile(*t, c->p.storage, npt);
    if (s) return s;
    c->tile = *t;
    c->tile.reserved = 0;
    fill_grid(c->g, c->p, c->tile);
    drop_graphs(c);
    return LBM_OK;
}

lbm_status lbm_get_tile(const lbm_ctx *c, lbm_tile *t) {
    if (!c || !t) return fail(LBM_ERR_INVALID_ARG, "null argument");
    *t = c->tile;
    return LBM_OK;
}

lbm_status lbm_autotune(lbm_ctx *c, int32_t trials, lbm_tile *best) {
    if (!c) return fail(LBM_ERR_INVALID_ARG, "ctx is NULL");
    if (trials < 1) return fail(LBM_ERR_INVALID_ARG, "trials < 1");
    std::vector<lbm_tile> cand;
    const int npt = npt_of(c->mode, c->p.storage);
    const int txs[] = {16, 32, 64, 128, 256};
    const int tys[] = {1, 2, 4, 8, 16, 32};
    const int czs[] = {4, 8, 16, 32, 64, 128};
    const int txmax = npt > 1 ? 256 : 128;
    auto add = [&](int tx, int ty, int cz) {
        lbm_tile t{tx, ty, std::min(cz, c->p.nz), 0};
        if (tx > txmax) return;
        if (t.tx > c->p.nx && t.tx != std::min(c->p.nx, txmax)) return;
        if (t.ty > c->p.ny) return;
        if ((t.tx / npt) * t.ty < 64) return;
        if ((c->mode == LBM_STEP_SPLIT ? check_split_tile(t, npt, c->p.storage) : check_tile(t, c->p.storage, npt)) !=
            LBM_OK)
            return;
        for (auto &o : cand)
            if (o.tx == t.tx && o.ty == t.ty && o.cz == t.cz) return;
        cand.push_back(t);
    };
    for (int tx : txs)
        for (int ty : tys)
            for (int cz : czs) add(std::min(tx, c->p.nx), ty, cz);
    if (cand.empty())
        cand.push_back(c->mode == LBM_STEP_SPLIT ? split_tile(c->p.nx, c->p.ny, c->p.nz, npt, c->p.storage)
                       : npt > 1           ? wide_tile(c->p.nx, c->p.ny, c->p.nz, npt)
                                           : default_tile(c->p.nx, c->p.ny, c->p.nz));
    g_err.clear();
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    lbm_status s = launch_walls(c, c->state());
    if (s) return s;
    float best_ms = 1e30f;
    lbm_tile bt = c->tile;
    for (const lbm_tile &t : cand) {
        GridDesc g{};
        fill_grid(g, c->p, t);
        if ((s = launch_step(c, g, c->state(), c->other(), npt))) return s;  // warm-up
        HIP_TRY(hipEventRecord(e0, c->stream));
        for (int k = 0; k < trials; ++k)
            if ((s = launch_step(c, g, c->state(), c->other(), npt))) return s;
        HIP_TRY(hipEventRecord(e1, c->stream));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
            best_ms = ms;
            bt = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->tile = bt;
    fill_grid(c->g, c->p, c->tile);
    drop_graphs(c);
    if (best) *best = bt;
    return LBM_OK;
}

lbm_status lbm_set_step_mode(lbm_ctx *c, int32_t mode, int32_t slab_planes) {
    if (!c) return fail(LBM_ERR_INVALID_ARG, "ctx is NULL");
    if (mode != LBM_STEP_FUSED && mode != LBM_STEP_SLABS && mode != LBM_STEP_PAIRS && mode != LBM_STEP_QUADS &&
        mode != LBM_STEP_SPLIT)
        return fail(LBM_ERR_INVALID_ARG, "unknown step mode %d", mode);
    if (slab_planes < 1) return fail(LBM_ERR_INVALID_ARG, "slab_planes < 1");
    if (mode == LBM_STEP_PAIRS) {
        if (c->p.storage == ST_F64) return fail(LBM_ERR_UNSUPPORTED, "pair mode needs FP32 or F16S storage");
        if (box_walls(c->p)) return fail(LBM_ERR_UNSUPPORTED, "runs with walls on x or y use their own kernel");
        if (c->p.nx % 2) return fail(LBM_ERR_UNSUPPORTED, "pair mode needs an even nx, got %d", c->p.nx);
    }
    if (mode == LBM_STEP_QUADS && !quads_apply(c->p))
        return fail(LBM_ERR_UNSUPPORTED, "quad mode needs F16S storage, nx a multiple of 4 (got %d) and no walls on x or y",
                    c->p.nx);
    if (c->p.storage == ST_F16N && mode != LBM_STEP_SPLIT)
        return fail(LBM_ERR_UNSUPPORTED, "F16N storage runs the split step only");
    if (mode == LBM_STEP_SPLIT && !split_apply(c->p))
        return fail(LBM_ERR_UNSUPPORTED, "split mode needs F16S or F16N storage with nx a multiple of 4 or FP32 with "
                    "even nx (got nx = %d), and no walls on x or y", c->p.nx);
    const int npt = npt_of(mode, c->p.storage);
    if (mode == LBM_STEP_SPLIT) {
        if (check_split_tile(c->tile, npt, c->p.storage) != LBM_OK) {
            g_err.clear();
            c->tile = split_tile(c->p.nx, c->p.ny, c->p.nz, npt, c->p.storage);
            fill_grid(c->g, c->p, c->tile);
        }
    } else if (check_tile(c->tile, c->p.storage, npt) != LBM_OK) {
        // The tile of the previous mode need not suit this one (a pair tile
        // 128 nodes wide needs 1024 threads at one node per thread).
        g_err.clear();
        c->tile = npt > 1 ? wide_tile(c->p.nx, c->p.ny, c->p.nz, npt) : default_tile(c->p.nx, c->p.ny, c->p.nz);
        fill_grid(c->g, c->p, c->tile);
    }
    c->mode = mode;
    c->slab = slab_planes;
    drop_graphs(c);
    return LBM_OK;
}

lbm_status lbm_get_step_mode(const lbm_ctx *c, int32_t *mode, int32_t *slab_planes) {
    if (!c || !mode) return fail(LBM_ERR_INVALID_ARG, "null argument");
    *mode = c->mode;
    if (slab_planes) *slab_planes = c->slab;
    return LBM_OK;
}

lbm_status lbm_set_write_check(lbm_ctx *c, int32_t enable) {
    if (!c) return fail(LBM_ERR_INVALID_ARG, "ctx is NULL");
    if (c->write_check != (enable != 0)) drop_graphs(c);
    c->write_check = enable != 0;
    return LBM_OK;
}

lbm_status lbm_set_store_policy(lbm_ctx *c, int32_t policy) {
    if (!c) return fail(LBM_ERR_INVALID_ARG, "ctx is NULL");
    if (policy != LBM_STORE_AUTO && policy != LBM_STORE_CACHED && policy != LBM_STORE_STREAM)
        return fail(LBM_ERR_INVALID_ARG, "unknown store policy %d", policy);
    if (c->store_policy != policy) drop_graphs(c);
    c->store_policy = policy;
    return LBM_OK;
}

lbm_status lbm_set_timing(lbm_ctx *c, int32_t enable) {
    if (!c) return fail(LBM_ERR_INVALID_ARG, "ctx is NULL");
    c->timing = enable != 0;
    c->nev = 0;
    return LBM_OK;
}

lbm_status lbm_kernel_time(lbm_ctx *c, double *avg_ms, int64_t *launches) {
    if (!c || !avg_ms) return fail(LBM_ERR_INVALID_ARG, "null argument");
    double tot = 0.0;
    if (c->nev) HIP_TRY(hipEventSynchronize(c->ev[2 * c->nev - 1]));
    for (size_t k = 0; k < c->nev; ++k) {
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
        tot += ms;
    }
    *avg_ms = c->nev ? tot / (double)c->nev : 0.0;
    if (launches) *launches = (int64_t)c->nev;
    c->nev = 0;
    return LBM_OK;
}

int64_t lbm_step_count(const lbm_ctx *c) { return c ? c->steps : -1; }

const char *lbm_status_string(lbm_status s) {
    switch (s) {
    case LBM_OK: return "ok";
    case LBM_ERR_INVALID_ARG: return "invalid argument";
    case LBM_ERR_BUFFER_TOO_SMALL: return "buffer too small";
    case LBM_ERR_HIP: return "HIP runtime error";
    case LBM_ERR_NONFINITE: return "non-finite populations";
    case LBM_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

const char *lbm_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched runs
// ---------------------------------------------------------------------------
struct lbm_batch {
    std::vector<lbm_ctx *> runs;
    std::vector<size_t> run_off;
    std::vector<RunDesc> desc;
    unsigned char *ws = nullptr;
    size_t desc_off = 0;
    int op = 0, storage = 0;
    int total_tiles = 0;
    int blocks = 0;
    int threads = 64;
    size_t smem = 0;
    int parity = 0;
    int item_nodes = 8192;
    int mode = LBM_STEP_FUSED;  // LBM_STEP_FUSED, LBM_STEP_PAIRS or LBM_STEP_SPLIT
    bool ring2 = false;         // split: some run's tile has a halo ring beyond the pullers
    int store_policy = LBM_STORE_AUTO;
    long long nodes = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    std::map<std::pair<int, int>, hipGraphExec_t> graphs;
    bool timing = true;
    std::vector<hipEvent_t> ev;
    size_t nev = 0;
    int64_t timed_steps = 0;
};

namespace {

lbm_tile batch_tile(const lbm_params &p, int item_nodes, int mode) {
    lbm_tile t{};
    if (mode == LBM_STEP_SPLIT) {  // whole rows up to 128 nodes, as many rows as the LDS takes
        const int npt = npt_of(mode, p.storage);
        t.tx = std::min(SPLIT_TX_DEFAULT, p.nx);
        t.ty = std::max(1, std::min(p.ny, split_rows(t.tx, npt, p.storage)));
        const int cols = t.tx * t.ty;
        t.cz = std::max(1, std::min(p.nz, (item_nodes + cols / 2) / cols));
        return t;
    }
    const bool pairs = mode == LBM_STEP_PAIRS;
    if (pairs) t.tx = std::min(p.nx, 128);
    else if (p.nx <= 128) t.tx = p.nx;
    else t.tx = default_tile(p.nx, p.ny, p.nz).tx;
    const int per_row = pairs ? t.tx / 2 : t.tx;
    t.ty = std::max(1, std::min(p.ny, STEP_MAX_THREADS / per_row));
    while (t.ty > 1 && block_threads(t.tx, t.ty, pairs ? 2 : 1) > STEP_MAX_THREADS) --t.ty;
    const int cols = t.tx * t.ty;
    t.cz = std::max(1, std::min(p.nz, (item_nodes + cols / 2) / cols));
    return t;
}

lbm_status batch_validate(const lbm_params *runs, int32_t n) {
    if (!runs || n < 1) return fail(LBM_ERR_INVALID_ARG, "need at least one run");
    for (int k = 0; k < n; ++k) {
        lbm_status s = validate(&runs[k]);
        if (s) return fail(s, "run %d: %s", k, g_err.c_str());
        if (runs[k].wall_z || runs[k].wall_x || runs[k].wall_y)
            return fail(LBM_ERR_UNSUPPORTED, "run %d: batched runs must be periodic", k);
        if (runs[k].op != runs[0].op || runs[k].storage != runs[0].storage)
            return fail(LBM_ERR_INVALID_ARG, "run %d: all runs must share op and storage", k);
    }
    return LBM_OK;
}

size_t batch_total(const lbm_params *runs, int32_t n, std::vector<size_t> *offs, size_t *desc_off) {
    size_t off = 0;
    for (int k = 0; k < n; ++k) {
        if (offs) offs->push_back(off);
        off += layout_of(runs[k]).total;
    }
    if (desc_off) *desc_off = off;
    off += align_up(sizeof(RunDesc) * (size_t)n);
    return off;
}

lbm_status batch_build(lbm_batch *b) {
    b->desc.assign(b->runs.size(), RunDesc{});
    b->ring2 = false;
    int tiles = 0;
    int threads = 64;
    size_t smem = 0;
    long long nodes = 0;
    for (size_t k = 0; k < b->runs.size(); ++k) {
        lbm_ctx *c = b->runs[k];
        c->tile = batch_tile(c->p, b->item_nodes, b->mode);
        fill_grid(c->g, c->p, c->tile);
        RunDesc &d = b->desc[k];
        d.g = c->g;
        d.pd = c->pd;
        d.offA = b->run_off[k] + c->L.A;
        d.offB = b->run_off[k] + c->L.B;
        d.tile_begin = tiles;
        tiles += c->g.ntiles;
        // F16N's pullers take the whole halo ring (see launch_step).
        if (b->mode == LBM_STEP_SPLIT && b->storage != ST_F16N && split_ring2(c->g.tx, c->g.ty)) b->ring2 = true;
        threads = b->mode == LBM_STEP_SPLIT ? 2 * SPLIT_ROLE
                                            : std::max(threads, block_threads(c->g.tx, c->g.ty, npt_of(b->mode, b->storage)));
        smem = b->mode == LBM_STEP_SPLIT ? 0 : std::max(smem, step_smem(c, c->g));
        nodes += c->g.N;
    }
    b->total_tiles = tiles;
    b->threads = threads;
    b->smem = smem;
    b->nodes = nodes;
    HIP_TRY(hipMemcpyAsync(b->ws + b->desc_off, b->desc.data(), sizeof(RunDesc) * b->desc.size(),
                           hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();
    return LBM_OK;
}

lbm_status batch_launch(lbm_batch *b, hipStream_t st, int parity, int blocks) {
    const RunDesc *d = reinterpret_cast<const RunDesc *>(b->ws + b->desc_off);
    const int nr = (int)b->runs.size();
    const bool nt = stream_stores(b->store_policy, b->desc_off);
#define LBM_SCASE(s, o, r2, n)                                                                                \
    if (b->storage == s && b->op == o && b->mode == LBM_STEP_SPLIT && b->ring2 == r2 && nt == n) {            \
        hipLaunchKernelGGL((k_batch_split<s, o, r2, n>), dim3(blocks), dim3(2 * SPLIT_ROLE), 0, st, b->ws, d,   \
                           nr, b->total_tiles, parity);                                                       \
        HIP_TRY(hipGetLastError());                                                                           \
        return LBM_OK;                                                                                        \
    }
#define LBM_SCASE4(s, o) LBM_SCASE(s, o, false, false) LBM_SCASE(s, o, true, false) \
    LBM_SCASE(s, o, false, true) LBM_SCASE(s, o, true, true)
    LBM_SCASE4(ST_F32, OP_NONORTH)
    LBM_SCASE4(ST_F32, OP_ORTH)
    LBM_SCASE4(ST_F16S, OP_NONORTH)
    LBM_SCASE4(ST_F16S, OP_ORTH)
    LBM_SCASE(ST_F16N, OP_NONORTH, false, false)
    LBM_SCASE(ST_F16N, OP_NONORTH, false, true)
    LBM_SCASE(ST_F16N, OP_ORTH, false, false)
    LBM_SCASE(ST_F16N, OP_ORTH, false, true)
#undef LBM_SCASE4
#undef LBM_SCASE
#define LBM_BCASE(s, o, pr)                                                                                   \
    if (b->storage == s && b->op == o && (b->mode == LBM_STEP_PAIRS) == pr && b->mode != LBM_STEP_SPLIT) {     \
        hipLaunchKernelGGL((k_batch_step<s, o, pr>), dim3(blocks), dim3(b->threads), b->smem, st, b->ws, d, nr, \
                           b->total_tiles, parity);                                                           \
        HIP_TRY(hipGetLastError());                                                                           \
        return LBM_OK;                                                                                        \
    }
    LBM_BCASE(ST_F64, OP_NONORTH, false)
    LBM_BCASE(ST_F64, OP_ORTH, false)
    LBM_BCASE(ST_F32, OP_NONORTH, false)
    LBM_BCASE(ST_F32, OP_ORTH, false)
    LBM_BCASE(ST_F16S, OP_NONORTH, false)
    LBM_BCASE(ST_F16S, OP_ORTH, false)
    LBM_BCASE(ST_F32, OP_NONORTH, true)
    LBM_BCASE(ST_F32, OP_ORTH, true)
    LBM_BCASE(ST_F16S, OP_NONORTH, true)
    LBM_BCASE(ST_F16S, OP_ORTH, true)
#undef LBM_BCASE
    return fail(LBM_ERR_UNSUPPORTED, "no batched kernel for storage %d op %d", b->storage, b->op);
}

bool batch_pairs_apply(const lbm_params *runs, int n) {
    for (int k = 0; k < n; ++k)
        if (!pairs_apply(runs[k])) return false;
    return true;
}

bool batch_split_apply(const lbm_batch *b) {
    for (lbm_ctx *c : b->runs)
        if (!split_apply(c->p)) return false;
    return true;
}

int default_blocks(const lbm_batch *b) {
    // Persistent grid: a few blocks per CU (one with the split step's LDS),
    // never more blocks than items.
    return std::max(1, std::min(b->total_tiles, b->mode == LBM_STEP_SPLIT ? 256 : 256 * 4));
}

void batch_advance(lbm_batch *b, int64_t n) {
    b->parity ^= (int)(n & 1);
    for (lbm_ctx *c : b->runs) {
        c->cur = b->parity;
        c->steps += n;
    }
}

lbm_status batch_event(lbm_batch *b, size_t k) {
    while (b->ev.size() <= k) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        b->ev.push_back(e);
    }
    HIP_TRY(hipEventRecord(b->ev[k], b->stream));
    return LBM_OK;
}

lbm_status batch_run(lbm_batch *b, lbm_ctx **out_run, int32_t run) {
    if (!b) return fail(LBM_ERR_INVALID_ARG, "batch is NULL");
    if (run < 0 || run >= (int)b->runs.size()) return fail(LBM_ERR_INVALID_ARG, "run %d out of range", run);
    *out_run = b->runs[run];
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_batch_workspace_bytes(const lbm_params *runs, int32_t n, size_t *bytes) {
    lbm_status s = batch_validate(runs, n);
    if (s) return s;
    if (!bytes) return fail(LBM_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = batch_total(runs, n, nullptr, nullptr);
    return LBM_OK;
}

lbm_status lbm_batch_create(const lbm_params *runs, int32_t n, void *dev_ws, size_t ws_bytes, void *hip_stream,
                            lbm_batch **out) {
    lbm_status s = batch_validate(runs, n);
    if (s) return s;
    if (!out || !dev_ws) return fail(LBM_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    if (reinterpret_cast<uintptr_t>(dev_ws) % kAlign)
        return fail(LBM_ERR_INVALID_ARG, "workspace must be %zu-byte aligned", kAlign);
    lbm_batch *b = new (std::nothrow) lbm_batch();
    if (!b) return fail(LBM_ERR_INVALID_ARG, "out of host memory");
    const size_t need = batch_total(runs, n, &b->run_off, &b->desc_off);
    if (ws_bytes < need) {
        delete b;
        return fail(LBM_ERR_BUFFER_TOO_SMALL, "workspace %zu bytes < required %zu", ws_bytes, need);
    }
    b->ws = static_cast<unsigned char *>(dev_ws);
    b->stream = static_cast<hipStream_t>(hip_stream);
    b->op = runs[0].op;
    b->storage = runs[0].storage;
    bool all_split = true;
    for (int k = 0; k < n; ++k) all_split = all_split && split_apply(runs[k]);
    b->mode = all_split ? LBM_STEP_SPLIT : batch_pairs_apply(runs, n) ? LBM_STEP_PAIRS : LBM_STEP_FUSED;
    for (int k = 0; k < n; ++k) {
        lbm_ctx *c = nullptr;
        s = lbm_create(&runs[k], b->ws + b->run_off[k], layout_of(runs[k]).total, hip_stream, &c);
        if (s) {
            lbm_batch_destroy(b);
            return s;
        }
        b->runs.push_back(c);
    }
    if ((s = batch_build(b))) {
        lbm_batch_destroy(b);
        return s;
    }
    b->blocks = default_blocks(b);
    *out = b;
    return LBM_OK;
}

lbm_status lbm_batch_destroy(lbm_batch *b) {
    if (!b) return fail(LBM_ERR_INVALID_ARG, "batch is NULL");
    for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
    for (lbm_ctx *c : b->runs) lbm_destroy(c);
    delete b;
    return LBM_OK;
}

lbm_status lbm_batch_init_droplets(lbm_batch *b, int32_t run, const lbm_droplet *d, int32_t n, double rho_L,
                                   double rho_V, double W) {
    lbm_ctx *c = nullptr;
    lbm_status s = batch_run(b, &c, run);
    if (s) return s;
    return lbm_init_droplets(c, d, n, rho_L, rho_V, W);
}

lbm_status lbm_batch_init_fields(lbm_batch *b, int32_t run, const double *rho, const double *u) {
    lbm_ctx *c = nullptr;
    lbm_status s = batch_run(b, &c, run);
    if (s) return s;
    return lbm_init_fields(c, rho, u);
}

lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps, int32_t graph_steps) {
    if (!b) return fail(LBM_ERR_INVALID_ARG, "batch is NULL");
    if (nsteps < 0 || graph_steps < 0) return fail(LBM_ERR_INVALID_ARG, "negative step count");
    lbm_status s;
    const size_t ev0 = 2 * b->nev;
    if (b->timing && nsteps > 0) {
        if ((s = batch_event(b, ev0))) return s;
    }
    int64_t left = nsteps;
    if (graph_steps > 0) {
        while (left >= graph_steps) {
            auto key = std::make_pair((int)graph_steps, b->parity);
            auto it = b->graphs.find(key);
            if (it == b->graphs.end()) {
                if (!b->cap) HIP_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
                HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
                for (int k = 0; k < graph_steps; ++k) {
                    s = batch_launch(b, b->cap, b->parity ^ (k & 1), b->blocks);
                    if (s) {
                        hipGraph_t g;
                        (void)hipStreamEndCapture(b->cap, &g);
                        return s;
                    }
                }
                hipGraph_t graph;
                HIP_TRY(hipStreamEndCapture(b->cap, &graph));
                hipGraphExec_t exec;
                hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e != hipSuccess) return fail(LBM_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
                it = b->graphs.emplace(key, exec).first;
            }
            HIP_TRY(hipGraphLaunch(it->second, b->stream));
            batch_advance(b, graph_steps);
            left -= graph_steps;
        }
    }
    for (; left > 0; --left) {
        if ((s = batch_launch(b, b->stream, b->parity, b->blocks))) return s;
        batch_advance(b, 1);
    }
    if (b->timing && nsteps > 0) {
        if ((s = batch_event(b, ev0 + 1))) return s;
        ++b->nev;
        b->timed_steps += nsteps;
    }
    return LBM_OK;
}

lbm_status lbm_batch_read_fields(lbm_batch *b, int32_t run, double *rho, double *u, double *p) {
    lbm_ctx *c = nullptr;
    lbm_status s = batch_run(b, &c, run);
    if (s) return s;
    return lbm_read_fields(c, rho, u, p);
}

lbm_status lbm_batch_read_populations(lbm_batch *b, int32_t run, double *f) {
    lbm_ctx *c = nullptr;
    lbm_status s = batch_run(b, &c, run);
    if (s) return s;
    return lbm_read_populations(c, f);
}

lbm_status lbm_batch_diagnostics(lbm_batch *b, int32_t run, const lbm_diag_request *req, lbm_diag *out) {
    lbm_ctx *c = nullptr;
    lbm_status s = batch_run(b, &c, run);
    if (s) return s;
    s = lbm_diagnostics(c, req, out);
    if (s == LBM_ERR_NONFINITE) return fail(s, "run %d: %s", run, g_err.c_str());
    return s;
}

lbm_status lbm_batch_status(lbm_batch *b, lbm_status *status) {
    if (!b || !status) return fail(LBM_ERR_INVALID_ARG, "null argument");
    int first = -1;
    int64_t first_bad = 0;
    for (size_t k = 0; k < b->runs.size(); ++k) {
        lbm_diag d{};
        const lbm_status s = lbm_diagnostics(b->runs[k], nullptr, &d);
        if (s != LBM_OK && s != LBM_ERR_NONFINITE) return s;
        status[k] = s;
        if (s == LBM_ERR_NONFINITE && first < 0) {
            first = (int)k;
            first_bad = d.nonfinite;
        }
    }
    if (first >= 0)
        return fail(LBM_ERR_NONFINITE, "run %d: %lld non-finite populations at step %lld", first,
                    (long long)first_bad, (long long)b->runs[first]->steps);
    return LBM_OK;
}

int32_t lbm_batch_runs(const lbm_batch *b) { return b ? (int32_t)b->runs.size() : 0; }

lbm_status lbm_batch_set_blocks(lbm_batch *b, int32_t blocks) {
    if (!b) return fail(LBM_ERR_INVALID_ARG, "batch is NULL");
    if (blocks < 1) return fail(LBM_ERR_INVALID_ARG, "blocks < 1");
    b->blocks = blocks;
    for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();
    return LBM_OK;
}

lbm_status lbm_batch_set_item_nodes(lbm_batch *b, int32_t item_nodes) {
    if (!b) return fail(LBM_ERR_INVALID_ARG, "batch is NULL");
    if (item_nodes < 1 || item_nodes > (1 << 24))
        return fail(LBM_ERR_INVALID_ARG, "item_nodes %d outside [1, 2^24]", item_nodes);
    b->item_nodes = item_nodes;
    lbm_status s = batch_build(b);
    if (s) return s;
    b->blocks = std::min(b->blocks, b->total_tiles);
    return LBM_OK;
}

lbm_status lbm_batch_get_tuning(const lbm_batch *b, int32_t *mode, int32_t *item_nodes, int32_t *blocks) {
    if (!b) return fail(LBM_ERR_INVALID_ARG, "batch is NULL");
    if (mode) *mode = b->mode;
    if (item_nodes) *item_nodes = b->item_nodes;
    if (blocks) *blocks = b->blocks;
    return LBM_OK;
}

lbm_status lbm_batch_set_step_mode(lbm_batch *b, int32_t mode) {
    if (!b) return fail(LBM_ERR_INVALID_ARG, "batch is NULL");
    if (mode != LBM_STEP_FUSED && mode != LBM_STEP_PAIRS && mode != LBM_STEP_SPLIT)
        return fail(LBM_ERR_INVALID_ARG, "batched runs take LBM_STEP_FUSED, LBM_STEP_PAIRS or LBM_STEP_SPLIT, got %d",
                    mode);
    if (mode == LBM_STEP_PAIRS) {
        for (size_t k = 0; k < b->runs.size(); ++k)
            if (!pairs_apply(b->runs[k]->p))
                return fail(LBM_ERR_UNSUPPORTED, "run %zu: pair mode needs FP32/F16S storage and even nx", k);
    }
    if (b->storage == ST_F16N && mode != LBM_STEP_SPLIT)
        return fail(LBM_ERR_UNSUPPORTED, "F16N storage runs the split step only");
    if (mode == LBM_STEP_SPLIT && !batch_split_apply(b))
        return fail(LBM_ERR_UNSUPPORTED, "split mode needs FP32 with even nx or F16S or F16N with nx a multiple of 4 in "
                    "every run");
    b->mode = mode;
    lbm_status s = batch_build(b);
    if (s) return s;
    b->blocks = std::min(mode == LBM_STEP_SPLIT ? 256 : b->blocks, b->total_tiles);
    return LBM_OK;
}

lbm_status lbm_batch_set_store_policy(lbm_batch *b, int32_t policy) {
    if (!b) return fail(LBM_ERR_INVALID_ARG, "batch is NULL");
    if (policy != LBM_STORE_AUTO && policy != LBM_STORE_CACHED && policy != LBM_STORE_STREAM)
        return fail(LBM_ERR_INVALID_ARG, "unknown store policy %d", policy);
    b->store_policy = policy;
    for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();
    return LBM_OK;
}

lbm_status lbm_batch_get_step_mode(const lbm_batch *b, int32_t *mode) {
    if (!b || !mode) return fail(LBM_ERR_INVALID_ARG, "null argument");
    *mode = b->mode;
    return LBM_OK;
}

lbm_status lbm_batch_autotune(lbm_batch *b, int32_t trials, int32_t *best_blocks) {
    if (!b) return fail(LBM_ERR_INVALID_ARG, "batch is NULL");
    if (trials < 1) return fail(LBM_ERR_INVALID_ARG, "trials < 1");
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int items[] = {4096, 8192, 16384, 32768};
    float best = 1e30f;
    int best_items = b->item_nodes, best_blk = b->blocks;
    int best_mode = b->mode;
    std::vector<int> modes;
    if (b->storage != ST_F16N) modes.push_back(LBM_STEP_FUSED);  // F16N runs the split step only
    bool all_pairs = true;
    for (lbm_ctx *c : b->runs) all_pairs = all_pairs && pairs_apply(c->p);
    if (all_pairs) modes.push_back(LBM_STEP_PAIRS);
    if (batch_split_apply(b)) modes.push_back(LBM_STEP_SPLIT);
    lbm_status s;
    for (int md : modes)
    for (int it : items) {
        b->mode = md;
        b->item_nodes = it;
        if ((s = batch_build(b))) return s;
        const int cands[] = {256, 512, 1024, 2048, 4096, b->total_tiles};
        for (int blk : cands) {
            if (blk > b->total_tiles) continue;
            if (md == LBM_STEP_SPLIT && blk > 256 && blk != b->total_tiles) continue;  // one block per CU
            // Steps write the other buffer of every run only: state unchanged.
            if ((s = batch_launch(b, b->stream, b->parity, blk))) return s;
            HIP_TRY(hipEventRecord(e0, b->stream));
            for (int k = 0; k < trials; ++k)
                if ((s = batch_launch(b, b->stream, b->parity, blk))) return s;
            HIP_TRY(hipEventRecord(e1, b->stream));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            if (ms < best) {
                best = ms;
                best_items = it;
                best_blk = blk;
                best_mode = md;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->mode = best_mode;
    b->item_nodes = best_items;
    if ((s = batch_build(b))) return s;
    b->blocks = best_blk;
    if (best_blocks) *best_blocks = best_blk;
    return LBM_OK;
}

lbm_status lbm_batch_kernel_time(lbm_batch *b, double *avg_ms, int64_t *launches) {
    if (!b || !avg_ms) return fail(LBM_ERR_INVALID_ARG, "null argument");
    double tot = 0.0;
    if (b->nev) HIP_TRY(hipEventSynchronize(b->ev[2 * b->nev - 1]));
    for (size_t k = 0; k < b->nev; ++k) {
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, b->ev[2 * k], b->ev[2 * k + 1]));
        tot += ms;
    }
    *avg_ms = b->timed_steps ? tot / (double)b->timed_steps : 0.0;
    if (launches) *launches = b->timed_steps;
    b->nev = 0;
    b->timed_steps = 0;
    return LBM_OK;
}

int64_t lbm_batch_nodes(const lbm_batch *b) { return b ? b->nodes : -1; }

}  // extern "C"
