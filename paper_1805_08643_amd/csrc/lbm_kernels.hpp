// HIP kernels of the D3Q19 MRT pseudopotential step for gfx950.
//
// Data layout in HBM: populations are structure-of-arrays, A[a * N + i] with
// i = (z * ny + y) * nx + x.  A holds post-collision values fbar*(x, t-1) at
// the node that produced them ("pull" form): the population that arrives at
// x in direction a is A[a][x - e_a] (Eq. (5) read backwards), or, across a
// half-way bounce-back wall, A[opp(a)][x].  Reads are shifted by +-1 in x
// (coalesced, one extra cache line per row), writes are aligned.
//
// The fused step (k_step) gives each block a tx x ty tile of (x, y) columns
// and a run of cz planes in z.  Marching up z, it pulls the 19 populations of
// the next plane, sums the density, evaluates psi and parks it in a four-plane
// LDS ring that also holds a one-node halo; the halo columns/rows pull their
// own populations (the density of a neighbour needs its full pull).  The
// interior populations of the next plane stay in registers and are collided
// one iteration later, once psi of the plane above is in LDS: HBM sees the
// 19 reads and 19 writes per node plus the halo and the two boundary planes
// of each z run.
#pragma once

#include "lbm_device.hpp"

namespace lbm {

struct GridDesc {
    int nx, ny, nz, wall;
    long long N;
    int tx, ty, cz;
    int ntx, nty, nzc;
    int ntiles, per_xcd;
};

__device__ inline int wrapi(int v, int n) {
    int r = v % n;
    return r < 0 ? r + n : r;
}

// Blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous run
// of tiles so that tiles sharing halo rows share an L2.
__device__ inline int xcd_tile(int b, int per_xcd) { return (b & 7) * per_xcd + (b >> 3); }

// Element at a 32-bit byte offset from a wave-uniform base: lets the
// compiler use the scalar-base + 32-bit vector-offset addressing form, so a
// lane carries one 32-bit offset per distinct row instead of 64-bit pointers.
template <class T> __device__ inline const T *at(const T *base, uint32_t boff) {
    return reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + boff);
}
template <class T> __device__ inline T *at(T *base, uint32_t boff) {
    return reinterpret_cast<T *>(reinterpret_cast<char *>(base) + boff);
}

// Pull the 19 populations arriving at (x, y, z).  Byte offsets of one
// direction plane must fit in 32 bits (N * sizeof(T) < 4 GiB).
template <int S, bool WALL>
__device__ inline void pull(const typename Storage<S>::T *__restrict__ A, size_t N, int nx, int ny,
                            int nz, int x, int xm, int xp, int y, int ym, int yp, int z,
                            const Phys<typename Storage<S>::R> &P, typename Storage<S>::R f[Q]) {
    using ST = Storage<S>;
    using T = typename ST::T;
    constexpr uint32_t E = sizeof(T);
    const bool bot = WALL && z == 0;
    const bool top = WALL && z == nz - 1;
    const int zm = WALL ? z - 1 : (z == 0 ? nz - 1 : z - 1);
    const int zq = WALL ? z + 1 : (z == nz - 1 ? 0 : z + 1);
    const uint32_t rowb = (uint32_t)nx * E;
    const uint32_t pc = (uint32_t)z * ny, pm = (uint32_t)zm * ny, pq = (uint32_t)zq * ny;
    const uint32_t r_c = (pc + y) * rowb, r_cm = (pc + ym) * rowb, r_cp = (pc + yp) * rowb;
    const uint32_t r_m = (pm + y) * rowb, r_mm = (pm + ym) * rowb, r_mp = (pm + yp) * rowb;
    const uint32_t r_q = (pq + y) * rowb, r_qm = (pq + ym) * rowb, r_qp = (pq + yp) * rowb;
    const uint32_t bx = (uint32_t)x * E, bxm = (uint32_t)xm * E, bxp = (uint32_t)xp * E;
    const uint32_t own = r_c + bx;
#define LBM_LD(d, boff) ST::load(at(A + (size_t)(d) * N, (boff)), P.sh(d), P.hsi)
    f[0] = LBM_LD(0, own);
    f[1] = LBM_LD(1, r_c + bxm);
    f[2] = LBM_LD(2, r_c + bxp);
    f[3] = LBM_LD(3, r_cm + bx);
    f[4] = LBM_LD(4, r_cp + bx);
    f[7] = LBM_LD(7, r_cm + bxm);
    f[8] = LBM_LD(8, r_cp + bxp);
    f[9] = LBM_LD(9, r_cp + bxm);
    f[10] = LBM_LD(10, r_cm + bxp);
    // e_z = +1 arrive from z - 1 (or bounce back at the bottom wall)
    f[5] = bot ? LBM_LD(6, own) : LBM_LD(5, r_m + bx);
    f[11] = bot ? LBM_LD(12, own) : LBM_LD(11, r_m + bxm);
    f[14] = bot ? LBM_LD(13, own) : LBM_LD(14, r_m + bxp);
    f[15] = bot ? LBM_LD(16, own) : LBM_LD(15, r_mm + bx);
    f[18] = bot ? LBM_LD(17, own) : LBM_LD(18, r_mp + bx);
    // e_z = -1 arrive from z + 1 (or bounce back at the top wall)
    f[6] = top ? LBM_LD(5, own) : LBM_LD(6, r_q + bx);
    f[12] = top ? LBM_LD(11, own) : LBM_LD(12, r_q + bxp);
    f[13] = top ? LBM_LD(14, own) : LBM_LD(13, r_q + bxm);
    f[16] = top ? LBM_LD(15, own) : LBM_LD(16, r_qp + bx);
    f[17] = top ? LBM_LD(18, own) : LBM_LD(17, r_qm + bx);
#undef LBM_LD
}

template <class R> __device__ inline R sum19(const R f[Q]) {
    // Same association as Pre::rho, so psi and the collision see one density.
    Pre<R> pr;
    pr.build(f);
    return pr.rho(f[0]);
}

// Interaction-force stencil of Eq. (15) on a psi ring: returns
// acc = sum_a w_a psi(x + e_a) e_a (w = 1/6 axis, 1/12 diagonal).
template <class R>
__device__ inline void psi_stencil(const R *__restrict__ lo, const R *__restrict__ mid,
                                   const R *__restrict__ hi, int c, int SX, R &ax, R &ay, R &az) {
    // planes: lo = z-1, mid = z, hi = z+1; c = LDS index of the node in a plane
    const R e = (R)(1.0 / 6.0), d = (R)(1.0 / 12.0);
    const R pxp = mid[c + 1], pxm = mid[c - 1], pyp = mid[c + SX], pym = mid[c - SX];
    const R pzp = hi[c], pzm = lo[c];
    const R ppx = mid[c + SX + 1], pmm = mid[c - SX - 1], ppm = mid[c - SX + 1], pmp = mid[c + SX - 1];
    const R hxp = hi[c + 1], hxm = hi[c - 1], hyp = hi[c + SX], hym = hi[c - SX];
    const R lxp = lo[c + 1], lxm = lo[c - 1], lyp = lo[c + SX], lym = lo[c - SX];
    // (1,1,0) ppx, (-1,-1,0) pmm, (1,-1,0) ppm, (-1,1,0) pmp
    // (1,0,1) hxp, (-1,0,-1) lxm, (1,0,-1) lxp, (-1,0,1) hxm
    // (0,1,1) hyp, (0,-1,-1) lym, (0,1,-1) lyp, (0,-1,1) hym
    ax = e * (pxp - pxm) + d * ((ppx - pmm) + (ppm - pmp) + (hxp - lxm) + (lxp - hxm));
    ay = e * (pyp - pym) + d * ((ppx - pmm) - (ppm - pmp) + (hyp - lym) + (lyp - hym));
    az = e * (pzp - pzm) + d * ((hxp - lxm) - (lxp - hxm) + (hyp - lym) - (lyp - hym));
}

// One block's z-march over a tile.  ps: LDS ring of 4 planes of
// (ty + 2) x (tx + 2) psi values.
template <int S, int OP, bool WALL>
__device__ inline void tile_march(const typename Storage<S>::T *__restrict__ A,
                                  typename Storage<S>::T *__restrict__ B,
                                  const typename Storage<S>::R *__restrict__ gpsi, const GridDesc &g,
                                  const Phys<typename Storage<S>::R> &P, int tile,
                                  typename Storage<S>::R *ps) {
    using ST = Storage<S>;
    using R = typename ST::R;
    const int TX = g.tx, TY = g.ty;
    const int SX = TX + 2, SP = (TY + 2) * SX;
    int t = tile;
    const int itx = t % g.ntx;
    t /= g.ntx;
    const int ity = t % g.nty;
    const int izc = t / g.nty;
    const int x0 = itx * TX, y0 = ity * TY;
    const int zb = izc * g.cz;
    const int ze = min(zb + g.cz, g.nz);
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const size_t N = (size_t)g.N;
    const int tid = threadIdx.x;

    // Interior column of this thread.
    const int lx = tid % TX, ly = tid / TX;
    const bool inner = ly < TY;
    const bool need_in = inner && lx <= nx - x0 && ly <= ny - y0;
    const bool active = inner && x0 + lx < nx && y0 + ly < ny;
    const int gx = wrapi(x0 + lx, nx), gy = wrapi(y0 + ly, ny);
    const int gxm = wrapi(gx - 1, nx), gxp = wrapi(gx + 1, nx);
    const int gym = wrapi(gy - 1, ny), gyp = wrapi(gy + 1, ny);
    const int cin = (ly + 1) * SX + lx + 1;

    // Halo ring position of this thread (top row, bottom row, left, right).
    const int nh = 2 * SX + 2 * TY;
    int hlx = -1, hly = -1;
    bool halo = false;
    if (tid < nh) {
        int h = tid;
        if (h < SX) {
            hlx = h - 1;
            hly = -1;
        } else if (h < 2 * SX) {
            hlx = h - SX - 1;
            hly = TY;
        } else if (h < 2 * SX + TY) {
            hlx = -1;
            hly = h - 2 * SX;
        } else {
            hlx = TX;
            hly = h - 2 * SX - TY;
        }
        halo = hlx <= nx - x0 && hly <= ny - y0;
    }
    const int hx = wrapi(x0 + hlx, nx), hy = wrapi(y0 + hly, ny);
    const int hxm = wrapi(hx - 1, nx), hxp = wrapi(hx + 1, nx);
    const int hym = wrapi(hy - 1, ny), hyp = wrapi(hy + 1, ny);
    const int chl = (hly + 1) * SX + hlx + 1;

    R fc[Q], fn[Q];
    R rc = (R)1, rn = (R)1;

    auto stage = [&](int zp, R *slot, R *fkeep, R &rkeep) {
        if (WALL && (zp < 0 || zp >= nz)) {
            const R *gp = gpsi + (zp < 0 ? 0 : (size_t)nx * ny);
            if (need_in) slot[cin] = gp[(size_t)gy * nx + gx];
            if (halo) slot[chl] = gp[(size_t)hy * nx + hx];
            return;
        }
        const int zw = WALL ? zp : wrapi(zp, nz);
        if (need_in) {
            pull<S, WALL>(A, N, nx, ny, nz, gx, gxm, gxp, gy, gym, gyp, zw, P, fkeep);
            rkeep = sum19<R>(fkeep);
            slot[cin] = pseudo_psi<R>(P, rkeep);
        }
        if (halo) {
            R fh[Q];
            pull<S, WALL>(A, N, nx, ny, nz, hx, hxm, hxp, hy, hym, hyp, zw, P, fh);
            slot[chl] = pseudo_psi<R>(P, sum19<R>(fh));
        }
    };

    auto slot_of = [&](int z) { return ps + ((z - zb + 1) & 3) * SP; };

    stage(zb - 1, slot_of(zb - 1), fn, rn);
    stage(zb, slot_of(zb), fc, rc);
    for (int z = zb; z < ze; ++z) {
        stage(z + 1, slot_of(z + 1), fn, rn);
        __syncthreads();
        if (active) {
            R ax, ay, az;
            const R *mid = slot_of(z);
            psi_stencil<R>(slot_of(z - 1), mid, slot_of(z + 1), cin, SX, ax, ay, az);
            const R mG_psi = -P.G * mid[cin];
            const R Fx = mG_psi * ax + rc * P.gx;
            const R Fy = mG_psi * ay + rc * P.gy;
            const R Fz = mG_psi * az + rc * P.gz;
            const R acc2 = ax * ax + ay * ay + az * az;
            collide<R, OP>(fc, rc, Fx, Fy, Fz, acc2, P);
            const uint32_t own = (((uint32_t)z * ny + gy) * nx + gx) * (uint32_t)sizeof(typename ST::T);
#pragma unroll
            for (int a = 0; a < Q; ++a) ST::store(at(B + (size_t)a * N, own), fc[a], P.sh(a), P.hs);
        }
#pragma unroll
        for (int a = 0; a < Q; ++a) fc[a] = fn[a];
        rc = rn;
    }
}

constexpr int STEP_MAX_THREADS = 512;

template <int S, int OP, bool WALL>
__global__ void __launch_bounds__(STEP_MAX_THREADS)
    k_step(const typename Storage<S>::T *__restrict__ A, typename Storage<S>::T *__restrict__ B,
           const typename Storage<S>::R *__restrict__ gpsi, GridDesc g, PhysD pd) {
    using R = typename Storage<S>::R;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R *ps = reinterpret_cast<R *>(smem_raw);
    const int tile = xcd_tile(blockIdx.x, g.per_xcd);
    if (tile >= g.ntiles) return;
    Phys<R> P;
    P.load(pd);
    tile_march<S, OP, WALL>(A, B, gpsi, g, P, tile, ps);
}

// ---------------------------------------------------------------------------
// Batched independent periodic runs.  One persistent launch per time step:
// every block walks a work list of (run, tile) items; item -> run by binary
// search over the runs' first-item indices.  Items are dealt so that each
// XCD takes a contiguous range (tiles of one run share halos through L2).
// ---------------------------------------------------------------------------
struct RunDesc {
    GridDesc g;
    PhysD pd;
    unsigned long long offA, offB;  // byte offsets of the two population buffers
    int tile_begin;
    int pad;
};

template <int S, int OP>
__global__ void __launch_bounds__(STEP_MAX_THREADS)
    k_batch_step(unsigned char *__restrict__ ws, const RunDesc *__restrict__ runs, int nruns, int total_tiles,
                 int parity) {
    using ST = Storage<S>;
    using T = typename ST::T;
    using R = typename ST::R;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R *ps = reinterpret_cast<R *>(smem_raw);
    const int per_xcd = (total_tiles + 7) / 8;
    const int nvirt = 8 * per_xcd;
    for (int v = blockIdx.x; v < nvirt; v += gridDim.x) {
        const int item = xcd_tile(v, per_xcd);
        if (item >= total_tiles) continue;
        int lo = 0, hi = nruns - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (runs[mid].tile_begin <= item) lo = mid;
            else hi = mid - 1;
        }
        const RunDesc &rd = runs[lo];
        const GridDesc g = rd.g;
        Phys<R> P;
        P.load(rd.pd);
        const T *src = reinterpret_cast<const T *>(ws + (parity ? rd.offB : rd.offA));
        T *dst = reinterpret_cast<T *>(ws + (parity ? rd.offA : rd.offB));
        tile_march<S, OP, false>(src, dst, nullptr, g, P, item - rd.tile_begin, ps);
        __syncthreads();  // the next item reuses the LDS ring
    }
}

// ---------------------------------------------------------------------------
// Wall support, Eq. (57): densities of the first two layers at each wall,
// then ghost psi one layer beyond each wall.
// rho_w planes: 0 -> z=0, 1 -> z=1, 2 -> z=nz-2, 3 -> z=nz-1.
// ---------------------------------------------------------------------------
template <int S>
__global__ void k_wall_rho(const typename Storage<S>::T *__restrict__ A,
                           typename Storage<S>::R *__restrict__ rho_w, GridDesc g, PhysD pd) {
    using R = typename Storage<S>::R;
    Phys<R> P;
    P.load(pd);
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const long long plane = (long long)nx * ny;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * plane) return;
    const int k = (int)(i / plane);
    const int rem = (int)(i - (long long)k * plane);
    const int x = rem % nx, y = rem / nx;
    const int z = k == 0 ? 0 : (k == 1 ? 1 : (k == 2 ? nz - 2 : nz - 1));
    R f[Q];
    pull<S, true>(A, (size_t)g.N, nx, ny, nz, x, wrapi(x - 1, nx), wrapi(x + 1, nx), y, wrapi(y - 1, ny),
                  wrapi(y + 1, ny), z, P, f);
    rho_w[i] = sum19<R>(f);
}

template <class R>
__global__ void k_ghost_psi(const R *__restrict__ rho_w, R *__restrict__ gpsi, GridDesc g, PhysD pd) {
    Phys<R> P;
    P.load(pd);
    const int nx = g.nx, ny = g.ny;
    const long long plane = (long long)nx * ny;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 2 * plane) return;
    const int side = (int)(i / plane);
    const int rem = (int)(i - side * plane);
    const int x = rem % nx, y = rem / nx;
    const R *l1 = rho_w + (side == 0 ? 0 : 3) * plane;  // first fluid layer
    const R *l2 = rho_w + (side == 0 ? 1 : 2) * plane;  // second fluid layer
    const R dx = l1[(size_t)y * nx + wrapi(x + 1, nx)] - l1[(size_t)y * nx + wrapi(x - 1, nx)];
    const R dy = l1[(size_t)wrapi(y + 1, ny) * nx + x] - l1[(size_t)wrapi(y - 1, ny) * nx + x];
    const R phi = r_sqrt(dx * dx + dy * dy);
    R rg = l2[rem] + phi * P.tan_wall;
    if (rg < P.ghost_rho_min) rg = P.ghost_rho_min;
    gpsi[i] = pseudo_psi<R>(P, rg);
}

// ---------------------------------------------------------------------------
// Whole-lattice psi (for readback and diagnostics; not on the step path).
// ---------------------------------------------------------------------------
template <int S, bool WALL>
__global__ void k_psi_full(const typename Storage<S>::T *__restrict__ A,
                           typename Storage<S>::R *__restrict__ psi, GridDesc g, PhysD pd) {
    using R = typename Storage<S>::R;
    Phys<R> P;
    P.load(pd);
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((long long)nx * ny));
        R f[Q];
        pull<S, WALL>(A, (size_t)g.N, nx, ny, nz, x, wrapi(x - 1, nx), wrapi(x + 1, nx), y, wrapi(y - 1, ny),
                      wrapi(y + 1, ny), z, P, f);
        psi[i] = pseudo_psi<R>(P, sum19<R>(f));
    }
}

template <class R>
__device__ inline R psi_at(const R *__restrict__ psi, const R *__restrict__ gpsi, const GridDesc &g, bool wall,
                           int x, int y, int z) {
    x = wrapi(x, g.nx);
    y = wrapi(y, g.ny);
    if (wall) {
        if (z < 0) return gpsi[(size_t)y * g.nx + x];
        if (z >= g.nz) return gpsi[(size_t)g.nx * g.ny + (size_t)y * g.nx + x];
    } else {
        z = wrapi(z, g.nz);
    }
    return psi[((size_t)z * g.ny + y) * g.nx + x];
}

// Node-level macroscopic quantities from the pulled populations and a psi field.
template <int S, bool WALL>
__device__ inline void node_macro(const typename Storage<S>::T *__restrict__ A,
                                  const typename Storage<S>::R *__restrict__ psi,
                                  const typename Storage<S>::R *__restrict__ gpsi, const GridDesc &g,
                                  const Phys<typename Storage<S>::R> &P, int x, int y, int z,
                                  typename Storage<S>::R &rho, typename Storage<S>::R u[3],
                                  typename Storage<S>::R j[3], typename Storage<S>::R F[3],
                                  typename Storage<S>::R &psi_c, bool &finite) {
    using R = typename Storage<S>::R;
    const int nx = g.nx, ny = g.ny;
    R f[Q];
    pull<S, WALL>(A, (size_t)g.N, nx, ny, g.nz, x, wrapi(x - 1, nx), wrapi(x + 1, nx), y, wrapi(y - 1, ny),
                  wrapi(y + 1, ny), z, P, f);
    finite = true;
#pragma unroll
    for (int a = 0; a < Q; ++a) finite = finite && isfinite(f[a]);
    Pre<R> pr;
    pr.build(f);
    rho = pr.rho(f[0]);
    j[0] = pr.jx();
    j[1] = pr.jy();
    j[2] = pr.jz();
    R acc[3] = {(R)0, (R)0, (R)0};
#pragma unroll
    for (int a = 1; a < Q; ++a) {
        const R w = a <= 6 ? (R)(1.0 / 6.0) : (R)(1.0 / 12.0);
        const R pn = psi_at<R>(psi, gpsi, g, WALL, x + ex(a), y + ey(a), z + ez(a));
        acc[0] += w * pn * (R)ex(a);
        acc[1] += w * pn * (R)ey(a);
        acc[2] += w * pn * (R)ez(a);
    }
    psi_c = psi[((size_t)z * ny + y) * nx + x];
    const R grav[3] = {P.gx, P.gy, P.gz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        F[d] = -P.G * psi_c * acc[d] + rho * grav[d];
        u[d] = (j[d] + (R)0.5 * F[d]) / rho;
    }
}

template <int S, bool WALL>
__global__ void k_fields(const typename Storage<S>::T *__restrict__ A, const typename Storage<S>::R *__restrict__ psi,
                         const typename Storage<S>::R *__restrict__ gpsi, double *__restrict__ rho_o,
                         double *__restrict__ u_o, double *__restrict__ p_o, GridDesc g, PhysD pd) {
    using R = typename Storage<S>::R;
    Phys<R> P;
    P.load(pd);
    const int nx = g.nx, ny = g.ny;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((long long)nx * ny));
        R rho, u[3], j[3], F[3], pc;
        bool fin;
        node_macro<S, WALL>(A, psi, gpsi, g, P, x, y, z, rho, u, j, F, pc, fin);
        if (rho_o) rho_o[i] = (double)rho;
        if (u_o) {
            u_o[i] = (double)u[0];
            u_o[g.N + i] = (double)u[1];
            u_o[2 * g.N + i] = (double)u[2];
        }
        if (p_o) p_o[i] = (double)(rho * (R)(1.0 / 3.0) + (R)0.5 * P.G * pc * pc);
    }
}

// Canonical populations out: f[a][i] = fbar_a(x, t).
template <int S, bool WALL>
__global__ void k_read_pops(const typename Storage<S>::T *__restrict__ A, double *__restrict__ f, GridDesc g,
                            PhysD pd) {
    using R = typename Storage<S>::R;
    Phys<R> P;
    P.load(pd);
    const int nx = g.nx, ny = g.ny;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((long long)nx * ny));
        R v[Q];
        pull<S, WALL>(A, (size_t)g.N, nx, ny, g.nz, x, wrapi(x - 1, nx), wrapi(x + 1, nx), y, wrapi(y - 1, ny),
                      wrapi(y + 1, ny), z, P, v);
#pragma unroll
        for (int a = 0; a < Q; ++a) f[(size_t)a * g.N + i] = (double)v[a];
    }
}

// Place canonical populations of node (x, y, z) into pull form: the value
// arriving in direction a lives at A[a][x - e_a], or at A[opp(a)][x] when
// x - e_a lies beyond a wall.
template <int S, bool WALL>
__device__ inline void scatter_node(typename Storage<S>::T *__restrict__ A, const GridDesc &g,
                                    const Phys<typename Storage<S>::R> &P, int x, int y, int z,
                                    const typename Storage<S>::R v[Q]) {
    using ST = Storage<S>;
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        int sz = z - ez(a);
        size_t idx;
        int d = a;
        if (WALL && (sz < 0 || sz >= g.nz)) {
            idx = ((size_t)z * g.ny + y) * g.nx + x;
            d = opp(a);
        } else {
            sz = wrapi(sz, g.nz);
            idx = ((size_t)sz * g.ny + wrapi(y - ey(a), g.ny)) * g.nx + wrapi(x - ex(a), g.nx);
        }
        ST::store(A + (size_t)d * g.N + idx, v[a], P.sh(a), P.hs);
    }
}

template <int S, bool WALL>
__global__ void k_write_pops(typename Storage<S>::T *__restrict__ A, const double *__restrict__ f, GridDesc g,
                             PhysD pd) {
    using R = typename Storage<S>::R;
    Phys<R> P;
    P.load(pd);
    const int nx = g.nx, ny = g.ny;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((long long)nx * ny));
        R v[Q];
#pragma unroll
        for (int a = 0; a < Q; ++a) v[a] = (R)f[(size_t)a * g.N + i];
        scatter_node<S, WALL>(A, g, P, x, y, z, v);
    }
}

template <int S, int OP, bool WALL>
__global__ void k_init_fields(typename Storage<S>::T *__restrict__ A, const double *__restrict__ rho,
                              const double *__restrict__ u, GridDesc g, PhysD pd) {
    using R = typename Storage<S>::R;
    Phys<R> P;
    P.load(pd);
    const int nx = g.nx, ny = g.ny;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((long long)nx * ny));
        R v[Q];
        equilibrium<R, OP>((R)rho[i], (R)u[i], (R)u[g.N + i], (R)u[2 * g.N + i], v);
        scatter_node<S, WALL>(A, g, P, x, y, z, v);
    }
}

struct DropletSet {
    double c[8][3];
    double r0[8];
    double u[8][3];
    int n;
    double rho_L, rho_V, W;
};

// Eq. (59) tanh profile per droplet; largest profile wins, velocity scaled by
// the liquid fraction.  Distances use the minimum image on periodic axes.
__device__ inline void droplet_rho_u(const DropletSet &D, const GridDesc &g, int x, int y, int z, double &rho,
                                     double u[3]) {
    double best = -1e300;
    int own = 0;
    for (int k = 0; k < D.n; ++k) {
        double d[3] = {x - D.c[k][0], y - D.c[k][1], z - D.c[k][2]};
        const int n[3] = {g.nx, g.ny, g.nz};
        for (int a = 0; a < 3; ++a) {
            if (a < 2 || !g.wall) {
                const double L = (double)n[a];
                double r = fmod(d[a] + 0.5 * L, L);
                if (r < 0) r += L;
                d[a] = r - 0.5 * L;
            }
        }
        const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double prof = 0.5 * (D.rho_L + D.rho_V) - 0.5 * (D.rho_L - D.rho_V) * tanh(2.0 * (r - D.r0[k]) / D.W);
        if (k == 0 || prof > best) {
            best = prof;
            own = k;
        }
    }
    rho = best;
    const double frac = (best - D.rho_V) / (D.rho_L - D.rho_V);
    for (int a = 0; a < 3; ++a) u[a] = D.u[own][a] * frac;
}

template <int S, int OP, bool WALL>
__global__ void k_init_droplets(typename Storage<S>::T *__restrict__ A, DropletSet D, GridDesc g, PhysD pd) {
    using R = typename Storage<S>::R;
    Phys<R> P;
    P.load(pd);
    const int nx = g.nx, ny = g.ny;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((long long)nx * ny));
        double rho, u[3];
        droplet_rho_u(D, g, x, y, z, rho, u);
        R v[Q];
        equilibrium<R, OP>((R)rho, (R)u[0], (R)u[1], (R)u[2], v);
        scatter_node<S, WALL>(A, g, P, x, y, z, v);
    }
}

// ---------------------------------------------------------------------------
// Diagnostics: per-block FP64 partials (fixed reduction tree), then one block
// adds the partials in block order.  Deterministic.
// ---------------------------------------------------------------------------
constexpr int NDIAG = 12;  // mass, mom x y z, max|u|, p_in, p_out, rho_in, rho_out, n_in, n_out, nonfinite
constexpr int DIAG_BLOCKS = 1024;
constexpr int DIAG_THREADS = 256;

struct DiagReq {
    double c[3];
    double r_in2, r_out2;
    int enabled;
};

template <class V> __device__ inline V wave_sum(V v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <class V> __device__ inline V wave_max(V v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

template <int S, bool WALL>
__global__ void __launch_bounds__(DIAG_THREADS)
    k_diag(const typename Storage<S>::T *__restrict__ A, const typename Storage<S>::R *__restrict__ psi,
           const typename Storage<S>::R *__restrict__ gpsi, double *__restrict__ partial, GridDesc g, PhysD pd,
           DiagReq rq) {
    using R = typename Storage<S>::R;
    Phys<R> P;
    P.load(pd);
    double acc[NDIAG];
#pragma unroll
    for (int k = 0; k < NDIAG; ++k) acc[k] = 0.0;
    const int nx = g.nx, ny = g.ny;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((long long)nx * ny));
        R rho, u[3], j[3], F[3], pc;
        bool fin;
        node_macro<S, WALL>(A, psi, gpsi, g, P, x, y, z, rho, u, j, F, pc, fin);
        acc[0] += (double)rho;
        for (int d = 0; d < 3; ++d) acc[1 + d] += (double)j[d] + 0.5 * (double)F[d];
        const double um = sqrt((double)(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
        acc[4] = fin ? fmax(acc[4], um) : acc[4];
        if (!fin) acc[11] += 1.0;
        if (rq.enabled) {
            const int n[3] = {g.nx, g.ny, g.nz};
            double d[3] = {x - rq.c[0], y - rq.c[1], z - rq.c[2]};
            for (int a = 0; a < 3; ++a) {
                if (a < 2 || !g.wall) {
                    const double L = (double)n[a];
                    double r = fmod(d[a] + 0.5 * L, L);
                    if (r < 0) r += L;
                    d[a] = r - 0.5 * L;
                }
            }
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            const double p = (double)rho / 3.0 + 0.5 * (double)P.G * (double)pc * (double)pc;
            if (r2 < rq.r_in2) {
                acc[5] += p;
                acc[7] += (double)rho;
                acc[9] += 1.0;
            } else if (r2 > rq.r_out2) {
                acc[6] += p;
                acc[8] += (double)rho;
                acc[10] += 1.0;
            }
        }
    }
    __shared__ double red[DIAG_THREADS / 64][NDIAG];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NDIAG; ++k) {
        const double v = (k == 4) ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (lane == 0) red[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < NDIAG) {
        const int k = threadIdx.x;
        double v = red[0][k];
        for (int w = 1; w < DIAG_THREADS / 64; ++w) v = (k == 4) ? fmax(v, red[w][k]) : v + red[w][k];
        partial[(size_t)blockIdx.x * NDIAG + k] = v;
    }
}

__global__ void k_diag_final(const double *__restrict__ partial, int nblocks, double *__restrict__ out) {
    const int k = threadIdx.x;
    if (k >= NDIAG) return;
    double v = 0.0;
    for (int b = 0; b < nblocks; ++b) v = (k == 4) ? fmax(v, partial[(size_t)b * NDIAG + k]) : v + partial[(size_t)b * NDIAG + k];
    out[k] = v;
}

}  // namespace lbm
