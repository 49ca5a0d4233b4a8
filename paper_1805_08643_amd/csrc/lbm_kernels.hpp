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

#include <type_traits>

#include "lbm_device.hpp"

namespace lbm {

struct GridDesc {
    int nx, ny, nz, wall;  // wall: half-way bounce-back walls in z
    long long N;
    int tx, ty, cz;
    int ntx, nty, nzc;
    int ntiles, per_xcd;
    int wall_x, wall_y;    // single-phase walls in x and y (moving lid on y = ny - 1/2)
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

// Byte offsets, within one z-plane of one direction, of the nine (y, x)
// neighbours a pull reads: computed once per thread; the plane part of every
// address is wave-uniform and lives in scalar registers.
struct NbOff {
    uint32_t c;             // (y, x)
    uint32_t xm, xp;        // (y, x-1), (y, x+1)
    uint32_t ym, yp;        // (y-1, x), (y+1, x)
    uint32_t mm, pp, pm, mp;  // (y-1, x-1), (y+1, x+1), (y+1, x-1), (y-1, x+1)
    __device__ inline void set(int x, int xm_, int xp_, int y, int ym_, int yp_, int nx, uint32_t E) {
        const uint32_t rb = (uint32_t)nx * E;
        const uint32_t ry = (uint32_t)y * rb, rym = (uint32_t)ym_ * rb, ryp = (uint32_t)yp_ * rb;
        const uint32_t bx = (uint32_t)x * E, bxm = (uint32_t)xm_ * E, bxp = (uint32_t)xp_ * E;
        c = ry + bx;
        xm = ry + bxm;
        xp = ry + bxp;
        ym = rym + bx;
        yp = ryp + bx;
        mm = rym + bxm;
        pp = ryp + bxp;
        pm = ryp + bxm;
        mp = rym + bxp;
    }
};

// Buffer descriptors over a population array: four groups of five direction
// planes (the last group has four, or five with the F16N reference plane), so
// every offset within a group fits the 32-bit scalar offset when
// 5 N sizeof(T) < 4 GiB.  Direction d lives in group d / 5 at scalar offset
// (d % 5) * N sizeof(T) + plane offset.
struct PopBuf {
    rsrc_t r[4];
    uint32_t dbytes;  // N * sizeof(T): bytes of one direction plane
    template <class T> __device__ inline void set(const T *base, size_t N, int planes = Q) {
        dbytes = (uint32_t)(N * sizeof(T));
        for (int k = 0; k < 4; ++k) {
            const int nd = k < 3 ? 5 : planes - 15;
            r[k] = make_rsrc(base + (size_t)(5 * k) * N, (uint32_t)nd * dbytes);
        }
    }
    __device__ inline rsrc_t of(int d) const { return r[d / 5]; }
    __device__ inline uint32_t so(int d, uint32_t plane) const { return (uint32_t)(d % 5) * dbytes + plane; }
};

// Pull the 19 populations arriving at the node with offsets o in plane z:
// direction a comes from (x - e_a), i.e. plane z - e_az, or, across a
// half-way bounce-back wall, from direction opp(a) at the node itself.
// PB = bytes of one z-plane of one direction.
// DEV (F16N): f receives the deviations h_a 2^-e from w_a rt (exact), and
// *rt the node's reference density.
template <int S, bool WALL, bool DEV = false>
__device__ inline void pull(const PopBuf &A, int nz, uint32_t PB, int z, const NbOff &o,
                            const Phys<typename Storage<S>::R> &P, typename Storage<S>::R f[Q],
                            float *rt = nullptr) {
    using ST = Storage<S>;
    static_assert(!DEV || S == ST_F16N, "deviation pull is F16N only");
    const bool bot = WALL && z == 0;
    const bool top = WALL && z == nz - 1;
    const int zm = WALL ? (bot ? z : z - 1) : (z == 0 ? nz - 1 : z - 1);
    const int zq = WALL ? (top ? z : z + 1) : (z == nz - 1 ? 0 : z + 1);
    const uint32_t pc = (uint32_t)z * PB, pm = (uint32_t)zm * PB, pq = (uint32_t)zq * PB;
    // F16N: every population arriving here is stored against this node's
    // reference density (plane 19 at the node).
    NodeShift ns;
    if constexpr (S == ST_F16N) {
        const float r = nref_val((uint16_t)__builtin_amdgcn_raw_buffer_load_b16(A.of(19), (int)o.c,
                                                                                (int)A.so(19, pc), LBM_BUF_AUX));
        if constexpr (DEV) *rt = r;
        else ns.set(r);
    }
    auto sh = [&](int d) {
        if constexpr (DEV) return 0.0f;
        else if constexpr (S == ST_F16N) return ns(d);
        else return P.sh(d);
    };
#define LBM_LD(d, plane, off) ST::ldb(A.of(d), (off), A.so((d), (plane)), sh(d), P.hsi)
    f[0] = LBM_LD(0, pc, o.c);
    f[1] = LBM_LD(1, pc, o.xm);
    f[2] = LBM_LD(2, pc, o.xp);
    f[3] = LBM_LD(3, pc, o.ym);
    f[4] = LBM_LD(4, pc, o.yp);
    f[7] = LBM_LD(7, pc, o.mm);
    f[8] = LBM_LD(8, pc, o.pp);
    f[9] = LBM_LD(9, pc, o.pm);
    f[10] = LBM_LD(10, pc, o.mp);
    if (!bot) {  // e_z = +1 arrive from z - 1
        f[5] = LBM_LD(5, pm, o.c);
        f[11] = LBM_LD(11, pm, o.xm);
        f[14] = LBM_LD(14, pm, o.xp);
        f[15] = LBM_LD(15, pm, o.ym);
        f[18] = LBM_LD(18, pm, o.yp);
    } else {  // bounce back at the bottom wall
        f[5] = LBM_LD(6, pc, o.c);
        f[11] = LBM_LD(12, pc, o.c);
        f[14] = LBM_LD(13, pc, o.c);
        f[15] = LBM_LD(16, pc, o.c);
        f[18] = LBM_LD(17, pc, o.c);
    }
    if (!top) {  // e_z = -1 arrive from z + 1
        f[6] = LBM_LD(6, pq, o.c);
        f[12] = LBM_LD(12, pq, o.xp);
        f[13] = LBM_LD(13, pq, o.xm);
        f[16] = LBM_LD(16, pq, o.yp);
        f[17] = LBM_LD(17, pq, o.ym);
    } else {  // bounce back at the top wall
        f[6] = LBM_LD(5, pc, o.c);
        f[12] = LBM_LD(11, pc, o.c);
        f[13] = LBM_LD(14, pc, o.c);
        f[16] = LBM_LD(15, pc, o.c);
        f[17] = LBM_LD(18, pc, o.c);
    }
#undef LBM_LD
}

// Where the population arriving at (x, y, z) in direction a is stored, with
// walls on any axis: (idx, d) of A, and whether it reflected off the moving
// face y = ny - 1/2 (then it carries lid_term(a) on top of the stored value).
__device__ inline void box_source(const GridDesc &g, int x, int y, int z, int a, size_t &idx, int &d, bool &lid) {
    int sx = x - ex(a), sy = y - ey(a), sz = z - ez(a);
    const bool out = (g.wall_x && (sx < 0 || sx >= g.nx)) || (g.wall_y && (sy < 0 || sy >= g.ny)) ||
                     (g.wall && (sz < 0 || sz >= g.nz));
    lid = out && g.wall_y && sy >= g.ny;
    if (out) {
        idx = ((size_t)z * g.ny + y) * g.nx + x;
        d = opp(a);
    } else {
        idx = ((size_t)wrapi(sz, g.nz) * g.ny + wrapi(sy, g.ny)) * g.nx + wrapi(sx, g.nx);
        d = a;
    }
}

// Moving-face term of a population arriving in direction a after reflection
// off y = ny - 1/2: +2 w_a lid_rho (e_a . lid_u) / c_s^2 (the sign of the
// term for the direction that hit the face is reversed, e_a = -e_hit).
template <class R> __device__ inline R lid_term(const Phys<R> &P, int a) {
    return (R)wclass(a) * ((R)ex(a) * P.lid6[0] + (R)ey(a) * P.lid6[1] + (R)ez(a) * P.lid6[2]);
}

template <int S>
__device__ inline void pull_box(const typename Storage<S>::T *__restrict__ A, const GridDesc &g, int x, int y,
                                int z, const Phys<typename Storage<S>::R> &P, typename Storage<S>::R f[Q]) {
    using ST = Storage<S>;
    NodeShift ns;
    if constexpr (S == ST_F16N) ns.set(nref_val(A[(size_t)19 * g.N + ((size_t)z * g.ny + y) * g.nx + x]));
#pragma unroll
    for (int a = 0; a < Q; ++a) {
        size_t idx;
        int d;
        bool lid;
        box_source(g, x, y, z, a, idx, d, lid);
        const typename Storage<S>::R sh = S == ST_F16N ? (typename Storage<S>::R)ns(a) : P.sh(a);
        f[a] = ST::load(A + (size_t)d * g.N + idx, sh, P.hsi);
        if (lid) f[a] += lid_term(P, a);
    }
}

// Pull at an arbitrary node (readback and diagnostics kernels).
template <int S, bool WALL>
__device__ inline void pull_at(const typename Storage<S>::T *__restrict__ A, const GridDesc &g, int x, int y, int z,
                               const Phys<typename Storage<S>::R> &P, typename Storage<S>::R f[Q]) {
    if (g.wall_x | g.wall_y) {
        pull_box<S>(A, g, x, y, z, P, f);
        return;
    }
    NbOff o;
    o.set(x, wrapi(x - 1, g.nx), wrapi(x + 1, g.nx), y, wrapi(y - 1, g.ny), wrapi(y + 1, g.ny), g.nx,
          (uint32_t)sizeof(typename Storage<S>::T));
    PopBuf pb;
    pb.set(A, (size_t)g.N, planes_of(S));
    pull<S, WALL>(pb, g.nz, (uint32_t)((size_t)g.nx * g.ny * sizeof(typename Storage<S>::T)), z, o, P, f);
}

template <class R> __device__ inline R sum19(const R f[Q]) {
    // Same association as Pre::rho, so psi and the collision see one density.
    Pre<R> pr;
    pr.build(f);
    return pr.rho(f[0]);
}

// F16N at an arbitrary node: the deviations h_a 2^-e from w_a rt (exact in
// FP32) into g; returns the node's reference rt.
template <bool WALL>
__device__ inline float pull_dev_at(const uint16_t *__restrict__ A, const GridDesc &g, int x, int y, int z,
                                    const Phys<float> &P, float g_[Q]) {
    NbOff o;
    o.set(x, wrapi(x - 1, g.nx), wrapi(x + 1, g.nx), y, wrapi(y - 1, g.ny), wrapi(y + 1, g.ny), g.nx,
          (uint32_t)sizeof(uint16_t));
    PopBuf pb;
    pb.set(A, (size_t)g.N, planes_of(ST_F16N));
    float rt;
    pull<ST_F16N, WALL, true>(pb, g.nz, (uint32_t)((size_t)g.nx * g.ny * sizeof(uint16_t)), z, o, P, g_, &rt);
    return rt;
}

// Density at an arbitrary node.  F16N: the node's reference plus the sum of
// its deviations, the density the split step computes.
template <int S, bool WALL>
__device__ inline typename Storage<S>::R density_at(const typename Storage<S>::T *__restrict__ A, const GridDesc &g,
                                                    int x, int y, int z, const Phys<typename Storage<S>::R> &P) {
    using R = typename Storage<S>::R;
    R f[Q];
    if constexpr (S == ST_F16N) {
        const float rt = pull_dev_at<WALL>(A, g, x, y, z, P, f);
        return rt + sum19<R>(f);
    } else {
        pull_at<S, WALL>(A, g, x, y, z, P, f);
        return sum19<R>(f);
    }
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

// Block barrier that orders LDS only: global loads issued before it (the
// prefetch of the next plane) and stores of the previous plane stay in
// flight across it.
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// One block's z-march over a tile.  ps: LDS ring of 4 planes of
// (ty + 2) x (tx + 2) psi values.
//
// Per plane z the block (i) pulls plane z+1 for its interior columns and its
// halo ring, all loads in flight together; (ii) turns the densities into psi
// in LDS; (iii) barriers; (iv) collides and stores plane z, whose
// populations were pulled one iteration earlier and stayed in registers.
// (Prefetching plane z+2 before the collision, for the whole tile or for the
// halo only, measured slower on MI355X.)
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
    const int cin = (ly + 1) * SX + lx + 1;
    constexpr uint32_t E = sizeof(typename ST::T);
    const uint32_t PB = (uint32_t)((size_t)nx * ny * E);  // bytes of one z-plane of one direction
    PopBuf bA, bB;
    bA.set(A, N);
    bB.set(B, N);
    NbOff oin;
    oin.set(gx, wrapi(gx - 1, nx), wrapi(gx + 1, nx), gy, wrapi(gy - 1, ny), wrapi(gy + 1, ny), nx, E);

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
    const int chl = (hly + 1) * SX + hlx + 1;
    NbOff oh;
    oh.set(hx, wrapi(hx - 1, nx), wrapi(hx + 1, nx), hy, wrapi(hy - 1, ny), wrapi(hy + 1, ny), nx, E);

    R fc[Q], fn[Q], fh[Q];
    R rc = (R)1, rn = (R)1;

    // Issue the loads of plane zp (interior into fi, halo into fhh).
    auto issue = [&](int zp, R *fi, R *fhh, bool do_in, bool do_halo) {
        if (WALL && (zp < 0 || zp >= nz)) return;
        const int zw = WALL ? zp : wrapi(zp, nz);
        if (do_in && need_in) pull<S, WALL>(bA, nz, PB, zw, oin, P, fi);
        if (do_halo && halo) pull<S, WALL>(bA, nz, PB, zw, oh, P, fhh);
    };
    // Densities and psi of plane zp into its LDS slot.
    auto finish = [&](int zp, R *slot, const R *fi, const R *fhh, R &rk, bool do_in, bool do_halo) {
        if (WALL && (zp < 0 || zp >= nz)) {
            const R *gp = gpsi + (zp < 0 ? 0 : (size_t)nx * ny);
            if (do_in && need_in) slot[cin] = gp[(size_t)gy * nx + gx];
            if (do_halo && halo) slot[chl] = gp[(size_t)hy * nx + hx];
            return;
        }
        if (do_in && need_in) {
            rk = sum19<R>(fi);
            slot[cin] = pseudo_psi<R>(P, rk);
        }
        if (do_halo && halo) slot[chl] = pseudo_psi<R>(P, sum19<R>(fhh));
    };
    auto slot_of = [&](int z) { return ps + ((z - zb + 1) & 3) * SP; };

    issue(zb - 1, fn, fh, true, true);
    finish(zb - 1, slot_of(zb - 1), fn, fh, rn, true, true);
    issue(zb, fc, fh, true, true);
    finish(zb, slot_of(zb), fc, fh, rc, true, true);
    for (int z = zb; z < ze; ++z) {
        issue(z + 1, fn, fh, true, true);
        finish(z + 1, slot_of(z + 1), fn, fh, rn, true, true);
        lds_barrier();
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
            const uint32_t pz = (uint32_t)z * PB;
#pragma unroll
            for (int a = 0; a < Q; ++a) ST::stb(fc[a], bB.of(a), oin.c, bB.so(a, pz), P.shh(a), P.hs);
        }
#pragma unroll
        for (int a = 0; a < Q; ++a) fc[a] = fn[a];
        rc = rn;
    }
}

#ifndef LBM_STEP_MAX_THREADS
#define LBM_STEP_MAX_THREADS 512
#endif
constexpr int STEP_MAX_THREADS = LBM_STEP_MAX_THREADS;
// Minimum waves per SIMD the step kernels are compiled for (register budget
// 512 / waves VGPRs); 0 leaves it to the launch bound.
#ifndef LBM_STEP_WAVES_PER_EU
#define LBM_STEP_WAVES_PER_EU 0
#endif
#if LBM_STEP_WAVES_PER_EU > 0
#define LBM_STEP_ATTR __launch_bounds__(STEP_MAX_THREADS) __attribute__((amdgpu_waves_per_eu(LBM_STEP_WAVES_PER_EU)))
#else
#define LBM_STEP_ATTR __launch_bounds__(STEP_MAX_THREADS)
#endif

template <int S, int OP, bool WALL>
__global__ void LBM_STEP_ATTR
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
// Two x-adjacent nodes per thread (FP32 and F16S storage, even nx).
//
// A thread owns nodes (xa, xa + 1) with xa even.  For every direction one
// wide access moves both values: 8 bytes for FP32, 4 for F16S.  Directions
// with e_x = 0 read an aligned pair; e_x = +1 reads the pair starting at
// xa - 1 and e_x = -1 the pair starting at xa + 1.  On the periodic seam
// (xa = 0 for e_x = +1, xa + 1 = nx - 1 for e_x = -1) the shifted pair would
// wrap: the lane reads the aligned pair instead and fetches the one wrapped
// value with a narrow load, in a branch only waves holding a seam lane take.
// The arithmetic per node is that of the one-node kernel, so the two give
// the same populations bit for bit.
// ---------------------------------------------------------------------------
template <int S> struct Wide;
template <> struct Wide<ST_F32> {
    using W = unsigned long long;  // two values
    using B = uint32_t;            // bits of one value
    __device__ static inline W ld(rsrc_t r, uint32_t vo, uint32_t so) {
        return __builtin_bit_cast(W, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, LBM_BUF_AUX));
    }
    __device__ static inline B one(rsrc_t r, uint32_t vo, uint32_t so) {
        return __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, LBM_BUF_AUX);
    }
    __device__ static inline B lo(W w) { return (B)w; }
    __device__ static inline B hi(W w) { return (B)(w >> 32); }
    __device__ static inline float cvt(B b, float, float) { return __uint_as_float(b); }
    __device__ static inline void st2(float a, float b, rsrc_t r, uint32_t vo, uint32_t so, float, float) {
        using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        const W w = (W)__float_as_uint(a) | ((W)__float_as_uint(b) << 32);
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, w), r, (int)vo, (int)so, LBM_BUF_STORE_AUX);
    }
};
template <> struct Wide<ST_F16S> {
    using W = uint32_t;
    using B = uint16_t;
    __device__ static inline W ld(rsrc_t r, uint32_t vo, uint32_t so) {
        return __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, LBM_BUF_AUX);
    }
    __device__ static inline B one(rsrc_t r, uint32_t vo, uint32_t so) {
        return __builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so, LBM_BUF_AUX);
    }
    __device__ static inline B lo(W w) { return (B)w; }
    __device__ static inline B hi(W w) { return (B)(w >> 16); }
    __device__ static inline float cvt(B b, float shift, float hsi) {
        return fmaf(__half2float(__ushort_as_half(b)), hsi, shift);
    }
    // Built as a two-lane half vector, the pair converts straight into the
    // low and high halves of one register (same roundings as two scalar
    // conversions, two instructions fewer than shifting and or-ing).
    using H2 = _Float16 __attribute__((ext_vector_type(2)));
    __device__ static inline void st2(float a, float b, rsrc_t r, uint32_t vo, uint32_t so, float shs, float hs) {
        const H2 h = {(_Float16)fmaf(a, hs, -shs), (_Float16)fmaf(b, hs, -shs)};
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, h), r, (int)vo, (int)so,
                                              LBM_BUF_STORE_AUX);
    }
};

// Byte offsets within one z-plane of one direction for a node pair.
struct NbOff2 {
    uint32_t c, ym, yp;    // aligned pair at xa, rows y, y-1, y+1
    uint32_t xm, mm, pm;   // pair from xa - 1 (xa on the seam), rows y, y-1, y+1
    uint32_t xp, mp, pp;   // pair from xa + 1 (xa on the seam), rows y, y-1, y+1
    uint32_t ry, rym, ryp; // row starts, for the wrapped value on the seam
    uint32_t xlast;        // (nx - 1) * sizeof(T)
    __device__ inline void set(int xa, bool wl, bool wr, int y, int ym_, int yp_, int nx, uint32_t E) {
        const uint32_t rb = (uint32_t)nx * E;
        ry = (uint32_t)y * rb;
        rym = (uint32_t)ym_ * rb;
        ryp = (uint32_t)yp_ * rb;
        const uint32_t b0 = (uint32_t)xa * E;
        const uint32_t bm = (uint32_t)(wl ? xa : xa - 1) * E;
        const uint32_t bp = (uint32_t)(wr ? xa : xa + 1) * E;
        c = ry + b0;
        ym = rym + b0;
        yp = ryp + b0;
        xm = ry + bm;
        mm = rym + bm;
        pm = ryp + bm;
        xp = ry + bp;
        mp = rym + bp;
        pp = ryp + bp;
        xlast = (uint32_t)(nx - 1) * E;
    }
};

// Pull of a node pair: fa for node xa, fb for node xa + 1.  wl: xa == 0;
// wr: xa + 1 == nx - 1 (the pair's shifted reads would cross the seam).
template <int S, bool WALL>
__device__ inline void pull2(const PopBuf &A, int nz, uint32_t PB, int z, const NbOff2 &o, bool wl, bool wr,
                             const Phys<typename Storage<S>::R> &P, typename Storage<S>::R fa[Q],
                             typename Storage<S>::R fb[Q]) {
    using WD = Wide<S>;
    using W = typename WD::W;
    using B = typename WD::B;
    const bool bot = WALL && z == 0;
    const bool top = WALL && z == nz - 1;
    const int zm = WALL ? (bot ? z : z - 1) : (z == 0 ? nz - 1 : z - 1);
    const int zq = WALL ? (top ? z : z + 1) : (z == nz - 1 ? 0 : z + 1);
    const uint32_t pc = (uint32_t)z * PB, pm = (uint32_t)zm * PB, pq = (uint32_t)zq * PB;
    W w[Q];
#define LBM_LW(i, d, plane, off) w[i] = WD::ld(A.of(d), (off), A.so((d), (plane)))
    LBM_LW(0, 0, pc, o.c);
    LBM_LW(1, 1, pc, o.xm);
    LBM_LW(2, 2, pc, o.xp);
    LBM_LW(3, 3, pc, o.ym);
    LBM_LW(4, 4, pc, o.yp);
    LBM_LW(7, 7, pc, o.mm);
    LBM_LW(8, 8, pc, o.pp);
    LBM_LW(9, 9, pc, o.pm);
    LBM_LW(10, 10, pc, o.mp);
    if (!bot) {
        LBM_LW(5, 5, pm, o.c);
        LBM_LW(11, 11, pm, o.xm);
        LBM_LW(14, 14, pm, o.xp);
        LBM_LW(15, 15, pm, o.ym);
        LBM_LW(18, 18, pm, o.yp);
    } else {
        LBM_LW(5, 6, pc, o.c);
        LBM_LW(11, 12, pc, o.c);
        LBM_LW(14, 13, pc, o.c);
        LBM_LW(15, 16, pc, o.c);
        LBM_LW(18, 17, pc, o.c);
    }
    if (!top) {
        LBM_LW(6, 6, pq, o.c);
        LBM_LW(12, 12, pq, o.xp);
        LBM_LW(13, 13, pq, o.xm);
        LBM_LW(16, 16, pq, o.yp);
        LBM_LW(17, 17, pq, o.ym);
    } else {
        LBM_LW(6, 5, pc, o.c);
        LBM_LW(12, 11, pc, o.c);
        LBM_LW(13, 14, pc, o.c);
        LBM_LW(16, 15, pc, o.c);
        LBM_LW(17, 18, pc, o.c);
    }
#undef LBM_LW
    // Seam values: e_x = +1 needs x = nx - 1 for node xa = 0; e_x = -1 needs
    // x = 0 for node xa + 1 = nx - 1.  Order: 1, 7, 9, 11, 13 / 2, 8, 10, 14, 12.
    B sl[5] = {0, 0, 0, 0, 0}, sr[5] = {0, 0, 0, 0, 0};
    if (wl) {
        sl[0] = WD::one(A.of(1), o.ry + o.xlast, A.so(1, pc));
        sl[1] = WD::one(A.of(7), o.rym + o.xlast, A.so(7, pc));
        sl[2] = WD::one(A.of(9), o.ryp + o.xlast, A.so(9, pc));
        if (!bot) sl[3] = WD::one(A.of(11), o.ry + o.xlast, A.so(11, pm));
        if (!top) sl[4] = WD::one(A.of(13), o.ry + o.xlast, A.so(13, pq));
    }
    if (wr) {
        sr[0] = WD::one(A.of(2), o.ry, A.so(2, pc));
        sr[1] = WD::one(A.of(8), o.ryp, A.so(8, pc));
        sr[2] = WD::one(A.of(10), o.rym, A.so(10, pc));
        if (!bot) sr[3] = WD::one(A.of(14), o.ry, A.so(14, pm));
        if (!top) sr[4] = WD::one(A.of(12), o.ry, A.so(12, pq));
    }
    // Unpack.  On the seam the aligned pair (xa, xa + 1) was read: for e_x =
    // +1 node xa + 1 takes the value at xa (its low half); for e_x = -1 node
    // xa takes the value at xa + 1 (its high half).
    auto plain = [&](int i) {
        fa[i] = WD::cvt(WD::lo(w[i]), P.sh(i), P.hsi);
        fb[i] = WD::cvt(WD::hi(w[i]), P.sh(i), P.hsi);
    };
    auto from_left = [&](int i, B seam, bool shifted) {  // e_x = +1
        const B a = wl && shifted ? seam : WD::lo(w[i]);
        const B b = wl && shifted ? WD::lo(w[i]) : WD::hi(w[i]);
        fa[i] = WD::cvt(a, P.sh(i), P.hsi);
        fb[i] = WD::cvt(b, P.sh(i), P.hsi);
    };
    auto from_right = [&](int i, B seam, bool shifted) {  // e_x = -1
        const B a = wr && shifted ? WD::hi(w[i]) : WD::lo(w[i]);
        const B b = wr && shifted ? seam : WD::hi(w[i]);
        fa[i] = WD::cvt(a, P.sh(i), P.hsi);
        fb[i] = WD::cvt(b, P.sh(i), P.hsi);
    };
    plain(0);
    plain(3);
    plain(4);
    plain(5);
    plain(6);
    plain(15);
    plain(16);
    plain(17);
    plain(18);
    from_left(1, sl[0], true);
    from_left(7, sl[1], true);
    from_left(9, sl[2], true);
    from_left(11, sl[3], !bot);
    from_left(13, sl[4], !top);
    from_right(2, sr[0], true);
    from_right(8, sr[1], true);
    from_right(10, sr[2], true);
    from_right(14, sr[3], !bot);
    from_right(12, sr[4], !top);
}

// z-march of a tile with two nodes per thread: tx nodes (even) by ty rows,
// (tx / 2) * ty interior threads; the halo ring is pulled one node per
// thread as in tile_march.
template <int S, int OP, bool WALL>
__device__ inline void tile_march2(const typename Storage<S>::T *__restrict__ A,
                                   typename Storage<S>::T *__restrict__ B,
                                   const typename Storage<S>::R *__restrict__ gpsi, const GridDesc &g,
                                   const Phys<typename Storage<S>::R> &P, int tile,
                                   typename Storage<S>::R *ps) {
    using ST = Storage<S>;
    using R = typename ST::R;
    using WD = Wide<S>;
    const int TX = g.tx, TY = g.ty, TXP = g.tx >> 1;
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

    // Interior pair of this thread: nodes x0 + 2 lx and x0 + 2 lx + 1.  A
    // pair starting at nx (a ragged last tile) supplies psi of the wrapped
    // columns 0 and 1 to the last real column.
    const int lx = tid % TXP, ly = tid / TXP;
    const bool inner = ly < TY;
    const int xa = x0 + 2 * lx;
    const bool need_in = inner && xa <= nx && ly <= ny - y0;
    const bool active = inner && xa < nx && y0 + ly < ny;
    const int gx = xa >= nx ? xa - nx : xa, gy = wrapi(y0 + ly, ny);
    const bool wl = gx == 0, wr = gx + 1 == nx - 1;
    const int cin = (ly + 1) * SX + 2 * lx + 1;
    constexpr uint32_t E = sizeof(typename ST::T);
    const uint32_t PB = (uint32_t)((size_t)nx * ny * E);
    PopBuf bA, bB;
    bA.set(A, N);
    bB.set(B, N);
    NbOff2 oin;
    oin.set(gx, wl, wr, gy, wrapi(gy - 1, ny), wrapi(gy + 1, ny), nx, E);

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
    const int chl = (hly + 1) * SX + hlx + 1;
    NbOff oh;
    oh.set(hx, wrapi(hx - 1, nx), wrapi(hx + 1, nx), hy, wrapi(hy - 1, ny), wrapi(hy + 1, ny), nx, E);

    R ca[Q], cb[Q], na[Q], nb[Q], fh[Q];
    R rca = (R)1, rcb = (R)1, rna = (R)1, rnb = (R)1;

    auto issue = [&](int zp, R *fa, R *fb) {
        if (WALL && (zp < 0 || zp >= nz)) return;
        const int zw = WALL ? zp : wrapi(zp, nz);
        if (need_in) pull2<S, WALL>(bA, nz, PB, zw, oin, wl, wr, P, fa, fb);
        if (halo) pull<S, WALL>(bA, nz, PB, zw, oh, P, fh);
    };
    auto finish = [&](int zp, R *slot, const R *fa, const R *fb, R &ra, R &rb) {
        if (WALL && (zp < 0 || zp >= nz)) {
            const R *gp = gpsi + (zp < 0 ? 0 : (size_t)nx * ny);
            if (need_in) {
                slot[cin] = gp[(size_t)gy * nx + gx];
                slot[cin + 1] = gp[(size_t)gy * nx + gx + 1];
            }
            if (halo) slot[chl] = gp[(size_t)hy * nx + hx];
            return;
        }
        if (need_in) {
            ra = sum19<R>(fa);
            rb = sum19<R>(fb);
            slot[cin] = pseudo_psi<R>(P, ra);
            slot[cin + 1] = pseudo_psi<R>(P, rb);
        }
        if (halo) slot[chl] = pseudo_psi<R>(P, sum19<R>(fh));
    };
    auto slot_of = [&](int z) { return ps + ((z - zb + 1) & 3) * SP; };

    issue(zb - 1, na, nb);
    finish(zb - 1, slot_of(zb - 1), na, nb, rna, rnb);
    issue(zb, ca, cb);
    finish(zb, slot_of(zb), ca, cb, rca, rcb);
    for (int z = zb; z < ze; ++z) {
        issue(z + 1, na, nb);
        finish(z + 1, slot_of(z + 1), na, nb, rna, rnb);
        lds_barrier();
        if (active) {
            const R *lo = slot_of(z - 1), *mid = slot_of(z), *hi = slot_of(z + 1);
            R ax, ay, az;
            psi_stencil<R>(lo, mid, hi, cin, SX, ax, ay, az);
            R mG_psi = -P.G * mid[cin];
            collide<R, OP>(ca, rca, mG_psi * ax + rca * P.gx, mG_psi * ay + rca * P.gy, mG_psi * az + rca * P.gz,
                           ax * ax + ay * ay + az * az, P);
            psi_stencil<R>(lo, mid, hi, cin + 1, SX, ax, ay, az);
            mG_psi = -P.G * mid[cin + 1];
            collide<R, OP>(cb, rcb, mG_psi * ax + rcb * P.gx, mG_psi * ay + rcb * P.gy, mG_psi * az + rcb * P.gz,
                           ax * ax + ay * ay + az * az, P);
            const uint32_t pz = (uint32_t)z * PB;
#pragma unroll
            for (int a = 0; a < Q; ++a) WD::st2(ca[a], cb[a], bB.of(a), oin.c, bB.so(a, pz), P.shh(a), P.hs);
        }
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            ca[a] = na[a];
            cb[a] = nb[a];
        }
        rca = rna;
        rcb = rnb;
    }
}

template <int S, int OP, bool WALL>
__global__ void LBM_STEP_ATTR
    k_step2(const typename Storage<S>::T *__restrict__ A, typename Storage<S>::T *__restrict__ B,
            const typename Storage<S>::R *__restrict__ gpsi, GridDesc g, PhysD pd) {
    using R = typename Storage<S>::R;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    R *ps = reinterpret_cast<R *>(smem_raw);
    const int tile = xcd_tile(blockIdx.x, g.per_xcd);
    if (tile >= g.ntiles) return;
    Phys<R> P;
    P.load(pd);
    tile_march2<S, OP, WALL>(A, B, gpsi, g, P, tile, ps);
}

// ---------------------------------------------------------------------------
// Eight-byte lanes: NPT x-adjacent nodes per thread in one 8-byte access per
// direction (NPT = 4 for F16S storage, 2 for FP32).
//
// Directions with e_x = 0 read the aligned group at xa; e_x = +1 reads the
// group starting at xa - 1 and e_x = -1 the one starting at xa + 1
// (unaligned 8-byte loads, which gfx950 serves).  On the periodic seam (xa =
// 0 for e_x = +1, xa + NPT - 1 = nx - 1 for e_x = -1) the lane reads the
// aligned group and fetches the one wrapped value with a narrow load; once
// the plane has arrived the wrapped value is shifted into the group, so that
// element k of every group is the value node k pulls.  Populations stay in
// storage format until a node is converted; the arithmetic per node is that
// of the one-node kernel, so the populations are the same bit for bit.
// ---------------------------------------------------------------------------
template <int S> struct Lane8;
template <> struct Lane8<ST_F16S> {
    static constexpr int NPT = 4, BITS = 16;
    using B = uint16_t;
    __device__ static inline B narrow(rsrc_t r, uint32_t vo, uint32_t so) {
        return (B)__builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so, LBM_BUF_AUX);
    }
    __device__ static inline float cvt(unsigned long long w, int k, float shift, float hsi) {
        return fmaf(__half2float(__ushort_as_half((uint16_t)(w >> (16 * k)))), hsi, shift);
    }
};
template <> struct Lane8<ST_F16N> : Lane8<ST_F16S> {};
template <> struct Lane8<ST_F32> {
    static constexpr int NPT = 2, BITS = 32;
    using B = uint32_t;
    __device__ static inline B narrow(rsrc_t r, uint32_t vo, uint32_t so) {
        return __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, LBM_BUF_AUX);
    }
    __device__ static inline float cvt(unsigned long long w, int k, float, float) {
        return __uint_as_float((uint32_t)(w >> (32 * k)));
    }
};

struct Wide8 {
    unsigned long long w[Q];  // NPT values per direction
};
template <int S> struct Seam8 {
    typename Lane8<S>::B sl[5], sr[5];  // wrapped seam values, left and right side
};

// Results of the NPT nodes of a group, packed per direction for one 8-byte
// store.  F16S converts straight into the halves of two registers.
template <int S> struct Out8;
template <> struct Out8<ST_F16S> {
    using H2 = _Float16 __attribute__((ext_vector_type(2)));
    H2 lo[Q], hi[Q];
    __device__ inline void put(int k, int a, float v, const Phys<float> &P) {
        const _Float16 h = (_Float16)fmaf(v, P.hs, -P.shh(a));
        if (k == 0) lo[a].x = h;
        else if (k == 1) lo[a].y = h;
        else if (k == 2) hi[a].x = h;
        else hi[a].y = h;
    }
    __device__ inline unsigned long long word(int a) const {
        return (unsigned long long)__builtin_bit_cast(uint32_t, lo[a]) |
               ((unsigned long long)__builtin_bit_cast(uint32_t, hi[a]) << 32);
    }
};
// F16N: values arrive dithered in FP32 and are truncated toward zero to
// binary16 (the stochastic rounding of the collider).  Out8<ST_F16N> keeps them
// and truncates two nodes per instruction at the store, for a loop over the
// group's nodes that the compiler unrolls (constant k); Out8Rolled truncates
// each at once and shifts it into bits 16k of the direction's word, for a loop
// kept rolled (k at run time).
template <> struct Out8<ST_F16N> {
    float y[Q][4];  // dithered FP32 values, truncated in pairs at the store
    __device__ inline void clear() {}
    __device__ inline void set_dithered(int k, int a, float v) { y[a][k] = v; }
    __device__ inline unsigned long long word(int a) const {
        return (unsigned long long)f16_trunc2(y[a][0], y[a][1]) | ((unsigned long long)f16_trunc2(y[a][2], y[a][3]) << 32);
    }
};
struct Out8Rolled {
    unsigned long long w[Q];
    __device__ inline void clear() {
#pragma unroll
        for (int a = 0; a < Q; ++a) w[a] = 0;
    }
    __device__ inline void set_dithered(int k, int a, float v) {
        w[a] |= (unsigned long long)(__builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(v, 0.0f)) & 0xFFFFu)
                << (16 * k);
    }
    __device__ inline unsigned long long word(int a) const { return w[a]; }
};
template <> struct Out8<ST_F32> {
    uint32_t lo[Q], hi[Q];
    __device__ inline void put(int k, int a, float v, const Phys<float> &) {
        if (k == 0) lo[a] = __float_as_uint(v);
        else hi[a] = __float_as_uint(v);
    }
    __device__ inline unsigned long long word(int a) const {
        return (unsigned long long)lo[a] | ((unsigned long long)hi[a] << 32);
    }
};

// Byte offsets within one z-plane of one direction for a node group.
template <int S> struct NbOff8 {
    uint32_t c, ym, yp;    // aligned group at xa, rows y, y-1, y+1
    uint32_t xm, mm, pm;   // group from xa - 1 (xa on the seam), rows y, y-1, y+1
    uint32_t xp, mp, pp;   // group from xa + 1 (xa + NPT - 1 on the seam), rows y, y-1, y+1
    uint32_t ry, rym, ryp; // row starts, for the wrapped value on the seam
    uint32_t xlast;        // (nx - 1) * sizeof(T)
    __device__ inline void set(int xa, bool wl, bool wr, int y, int ym_, int yp_, int nx) {
        constexpr uint32_t E = sizeof(typename Storage<S>::T);
        const uint32_t rb = (uint32_t)nx * E;
        ry = (uint32_t)y * rb;
        rym = (uint32_t)ym_ * rb;
        ryp = (uint32_t)yp_ * rb;
        const uint32_t b0 = (uint32_t)xa * E;
        const uint32_t bm = (uint32_t)(wl ? xa : xa - 1) * E;
        const uint32_t bp = (uint32_t)(wr ? xa : xa + 1) * E;
        c = ry + b0;
        ym = rym + b0;
        yp = ryp + b0;
        xm = ry + bm;
        mm = rym + bm;
        pm = ryp + bm;
        xp = ry + bp;
        mp = rym + bp;
        pp = ryp + bp;
        xlast = (uint32_t)(nx - 1) * E;
    }
};

__device__ inline uint32_t u_so(const PopBuf &A, int d, uint32_t plane) {
    return __builtin_amdgcn_readfirstlane(A.so(d, plane));
}

// Issue the loads of a node group at plane z (wl: xa == 0; wr: xa + NPT - 1
// == nx - 1).
template <int S, bool WALL>
__device__ inline void load8(const PopBuf &A, int nz, uint32_t PB, int z, const NbOff8<S> &o, Wide8 &r,
                             Seam8<S> &sm) {
    using L = Lane8<S>;
    const bool bot = WALL && z == 0;
    const bool top = WALL && z == nz - 1;
    const int zm = WALL ? (bot ? z : z - 1) : (z == 0 ? nz - 1 : z - 1);
    const int zq = WALL ? (top ? z : z + 1) : (z == nz - 1 ? 0 : z + 1);
    const uint32_t pc = __builtin_amdgcn_readfirstlane((uint32_t)z * PB);
    const uint32_t pm = __builtin_amdgcn_readfirstlane((uint32_t)zm * PB);
    const uint32_t pq = __builtin_amdgcn_readfirstlane((uint32_t)zq * PB);
#define LBM_LQ(i, d, plane, off)                                                                               \
    r.w[i] = __builtin_bit_cast(unsigned long long,                                                         \
                                __builtin_amdgcn_raw_buffer_load_b64(A.of(d), (int)(off), (int)u_so(A, d, plane), \
                                                                     LBM_BUF_AUX))
    LBM_LQ(0, 0, pc, o.c);
    LBM_LQ(1, 1, pc, o.xm);
    LBM_LQ(2, 2, pc, o.xp);
    LBM_LQ(3, 3, pc, o.ym);
    LBM_LQ(4, 4, pc, o.yp);
    LBM_LQ(7, 7, pc, o.mm);
    LBM_LQ(8, 8, pc, o.pp);
    LBM_LQ(9, 9, pc, o.pm);
    LBM_LQ(10, 10, pc, o.mp);
    if (!bot) {
        LBM_LQ(5, 5, pm, o.c);
        LBM_LQ(11, 11, pm, o.xm);
        LBM_LQ(14, 14, pm, o.xp);
        LBM_LQ(15, 15, pm, o.ym);
        LBM_LQ(18, 18, pm, o.yp);
    } else {
        LBM_LQ(5, 6, pc, o.c);
        LBM_LQ(11, 12, pc, o.c);
        LBM_LQ(14, 13, pc, o.c);
        LBM_LQ(15, 16, pc, o.c);
        LBM_LQ(18, 17, pc, o.c);
    }
    if (!top) {
        LBM_LQ(6, 6, pq, o.c);
        LBM_LQ(12, 12, pq, o.xp);
        LBM_LQ(13, 13, pq, o.xm);
        LBM_LQ(16, 16, pq, o.yp);
        LBM_LQ(17, 17, pq, o.ym);
    } else {
        LBM_LQ(6, 5, pc, o.c);
        LBM_LQ(12, 11, pc, o.c);
        LBM_LQ(13, 14, pc, o.c);
        LBM_LQ(16, 15, pc, o.c);
        LBM_LQ(17, 18, pc, o.c);
    }
#undef LBM_LQ
    // Every lane issues the ten seam loads (from valid addresses; only seam
    // lanes use the values), so each wave issues the same loads in the same
    // order and the wait counts need no merging across branches.
    const uint32_t pmb = bot ? pc : pm, pqt = top ? pc : pq;
    sm.sl[0] = L::narrow(A.of(1), o.ry + o.xlast, u_so(A, 1, pc));  // order 1, 7, 9, 11, 13: value at x = nx - 1
    sm.sl[1] = L::narrow(A.of(7), o.rym + o.xlast, u_so(A, 7, pc));
    sm.sl[2] = L::narrow(A.of(9), o.ryp + o.xlast, u_so(A, 9, pc));
    sm.sl[3] = L::narrow(A.of(11), o.ry + o.xlast, u_so(A, 11, pmb));
    sm.sl[4] = L::narrow(A.of(13), o.ry + o.xlast, u_so(A, 13, pqt));
    sm.sr[0] = L::narrow(A.of(2), o.ry, u_so(A, 2, pc));  // order 2, 8, 10, 14, 12: value at x = 0
    sm.sr[1] = L::narrow(A.of(8), o.ryp, u_so(A, 8, pc));
    sm.sr[2] = L::narrow(A.of(10), o.rym, u_so(A, 10, pc));
    sm.sr[3] = L::narrow(A.of(14), o.ry, u_so(A, 14, pmb));
    sm.sr[4] = L::narrow(A.of(12), o.ry, u_so(A, 12, pqt));
}

// Once the loads of a plane have arrived, seam lanes shift the wrapped value
// into the groups of the shifted directions.
template <int S, bool WALL>
__device__ inline void fold8(Wide8 &r, const Seam8<S> &sm, int nz, int z, bool wl, bool wr) {
    constexpr int BITS = Lane8<S>::BITS;
    const bool bot = WALL && z == 0;
    const bool top = WALL && z == nz - 1;
    auto left = [&](int i, int s) {  // e_x = +1: (seam, g0, .., g_{NPT-2})
        const unsigned long long v = (r.w[i] << BITS) | (unsigned long long)sm.sl[s];
        r.w[i] = wl ? v : r.w[i];
    };
    auto right = [&](int i, int s) {  // e_x = -1: (g1, .., g_{NPT-1}, seam)
        const unsigned long long v = (r.w[i] >> BITS) | ((unsigned long long)sm.sr[s] << (64 - BITS));
        r.w[i] = wr ? v : r.w[i];
    };
    left(1, 0);
    left(7, 1);
    left(9, 2);
    if (!bot) left(11, 3);
    if (!top) left(13, 4);
    right(2, 0);
    right(8, 1);
    right(10, 2);
    if (!bot) right(14, 3);
    if (!top) right(12, 4);
}

// Populations of node k of a folded group, converted to FP32.
template <int S> __device__ inline void unpack8(const Wide8 &r, int k, const Phys<float> &P, float f[Q]) {
#pragma unroll
    for (int a = 0; a < Q; ++a) f[a] = Lane8<S>::cvt(r.w[a], k, P.sh(a), P.hsi);
}
// F16N: node k's deviations g_a = h_a 2^-e from w_a rt (exact in FP32); rt
// is element k of the group's reference word (plane 19 at the group).
__device__ inline void unpack8n(const Wide8 &r, int k, const Phys<float> &P, float g[Q]) {
#pragma unroll
    for (int a = 0; a < Q; ++a) g[a] = Lane8<ST_F16N>::cvt(r.w[a], k, 0.0f, P.hsi);
}
__device__ inline float ref_of(unsigned long long rw, int k) { return nref_val((uint16_t)(rw >> (16 * k))); }

// z-march of a tile with four nodes per thread: tx nodes (a multiple of 4)
// by ty rows, (tx / 4) * ty interior threads; the halo ring is pulled one
// node per thread as in tile_march.
template <int OP, bool WALL>
__device__ inline void tile_march4(const uint16_t *__restrict__ A, uint16_t *__restrict__ B,
                                   const float *__restrict__ gpsi, const GridDesc &g, const Phys<float> &P,
                                   int tile, float *ps) {
    using R = float;
    const int TX = g.tx, TY = g.ty, TXQ = g.tx >> 2;
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

    // Interior quad of this thread: nodes x0 + 4 lx .. x0 + 4 lx + 3.  A quad
    // starting at nx (a ragged last tile) supplies psi of the wrapped columns
    // 0..3 to the last real column.
    const int lx = tid % TXQ, ly = tid / TXQ;
    const bool inner = ly < TY;
    const int xa = x0 + 4 * lx;
    const bool need_in = inner && xa <= nx && ly <= ny - y0;
    const bool active = inner && xa < nx && y0 + ly < ny;
    const int gx = xa >= nx ? xa - nx : xa, gy = wrapi(y0 + ly, ny);
    const bool wl = gx == 0, wr = gx + 3 == nx - 1;
    const int cin = (ly + 1) * SX + 4 * lx + 1;
    constexpr uint32_t E = 2;
    const uint32_t PB = (uint32_t)((size_t)nx * ny * E);
    PopBuf bA, bB;
    bA.set(A, N);
    bB.set(B, N);
    NbOff8<ST_F16S> oin;
    oin.set(gx, wl, wr, gy, wrapi(gy - 1, ny), wrapi(gy + 1, ny), nx);

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
    const int chl = (hly + 1) * SX + hlx + 1;
    NbOff oh;
    oh.set(hx, wrapi(hx - 1, nx), wrapi(hx + 1, nx), hy, wrapi(hy - 1, ny), wrapi(hy + 1, ny), nx, E);

    Wide8 cq, nq;  // planes z and z + 1, storage format
    R rc[4] = {1, 1, 1, 1}, rn[4] = {1, 1, 1, 1};
    auto zwrap = [&](int zp) { return WALL ? zp : wrapi(zp, nz); };
    auto slot_of = [&](int z) { return ps + ((z - zb + 1) & 3) * SP; };
    // Pull plane zp into q and put its psi in LDS; densities into rho.
    auto pull_plane = [&](int zp, Wide8 &q, R *rho) {
        R *slot = slot_of(zp);
        if (WALL && (zp < 0 || zp >= nz)) {
            const R *gp = gpsi + (zp < 0 ? 0 : (size_t)nx * ny);
            if (need_in) {
#pragma unroll
                for (int k = 0; k < 4; ++k) slot[cin + k] = gp[(size_t)gy * nx + gx + k];
            }
            if (halo) slot[chl] = gp[(size_t)hy * nx + hx];
            return;
        }
        const int zw = zwrap(zp);
        // Interior loads, conversions and psi run on every lane (lanes
        // without a pair of their own read valid nodes and keep the result
        // to themselves), so the loads are consumed on the path that issued
        // them; the halo node's loads likewise.
        Seam8<ST_F16S> sm;
        load8<ST_F16S, WALL>(bA, nz, PB, zw, oin, q, sm);
        if (halo) {
            R fh[Q];
            pull<ST_F16S, WALL>(bA, nz, PB, zw, oh, P, fh);
            slot[chl] = pseudo_psi<R>(P, sum19<R>(fh));
        }
        fold8<ST_F16S, WALL>(q, sm, nz, zw, wl, wr);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            R f[Q];
            unpack8<ST_F16S>(q, k, P, f);
            rho[k] = sum19<R>(f);
            const R p = pseudo_psi<R>(P, rho[k]);
            if (need_in) slot[cin + k] = p;
        }
    };

    pull_plane(zb - 1, nq, rn);
    pull_plane(zb, cq, rc);
    for (int z = zb; z < ze; ++z) {
        pull_plane(z + 1, nq, rn);
        lds_barrier();
        if (active) {
            const R *lo = slot_of(z - 1), *mid = slot_of(z), *hi = slot_of(z + 1);
            Out8<ST_F16S> out;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                R f[Q];
                unpack8<ST_F16S>(cq, k, P, f);
                R ax, ay, az;
                psi_stencil<R>(lo, mid, hi, cin + k, SX, ax, ay, az);
                const R rho = rc[k];
                const R mG_psi = -P.G * mid[cin + k];
                collide<R, OP>(f, rho, mG_psi * ax + rho * P.gx, mG_psi * ay + rho * P.gy, mG_psi * az + rho * P.gz,
                               ax * ax + ay * ay + az * az, P);
#pragma unroll
                for (int a = 0; a < Q; ++a) out.put(k, a, f[a], P);
            }
            const uint32_t pz = __builtin_amdgcn_readfirstlane((uint32_t)z * PB);
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(bB.of(a), 0, 0, 0));
                __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, out.word(a)), bB.of(a), (int)oin.c,
                                                      (int)u_so(bB, a, pz), LBM_BUF_STORE_AUX);
            }
        }
        cq = nq;
#pragma unroll
        for (int k = 0; k < 4; ++k) rc[k] = rn[k];
    }
}

template <int OP, bool WALL>
__global__ void LBM_STEP_ATTR k_step4(const uint16_t *__restrict__ A, uint16_t *__restrict__ B,
                                      const float *__restrict__ gpsi, GridDesc g, PhysD pd) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float *ps = reinterpret_cast<float *>(smem_raw);
    const int tile = xcd_tile(blockIdx.x, g.per_xcd);
    if (tile >= g.ntiles) return;
    Phys<float> P;
    P.load(pd);
    tile_march4<OP, WALL>(A, B, gpsi, g, P, tile, ps);
}

// ---------------------------------------------------------------------------
// Split step: pulling and colliding waves (FP32 and F16S, eight-byte lanes).
//
// A 512-thread block splits into two roles by wave.  Waves 0-3 pull planes:
// global loads, psi into the LDS ring, populations (storage format) and
// densities into LDS.  Waves 4-7 collide planes from LDS and store them.  The pullers
// run three planes ahead of the colliders, so on every SIMD one wave waits on
// memory while the other computes and the two phases overlap instead of
// alternating.  One barrier per plane; both roles run the same
// number of iterations.  Tiles hold at most SPLIT_ROLE groups of NPT nodes
// (128 x 8 nodes for F16S, 128 x 4 for FP32), so that three planes of
// populations fit in LDS.  Per-node arithmetic is that of the one-node
// kernel: the same populations bit for bit.
// ---------------------------------------------------------------------------
constexpr int SPLIT_TX = 256, SPLIT_TY = 8, SPLIT_ROLE = 256;  // max tile width / default rows, threads per role
constexpr int SPLIT_SP = 6 * (SPLIT_TX + 2);                    // psi ring slot: (tx + 2)(ty + 2) <= 256 x 4 + ring
constexpr int SPLIT_NODES = 1024;                               // max nodes per tile plane

template <int S> struct SplitLds {
    unsigned long long qbuf[3][Q][SPLIT_ROLE];  // populations of three planes, one group per slot
    float rbuf[3][SPLIT_NODES];                 // densities of three planes
    float ring[4][SPLIT_SP];                    // psi ring
};
// F16N adds a ring of this step's binary16 densities (with the halo): the
// references of the populations the colliders store, each for the node that
// will pull it.  To stay within the 160 KiB of LDS its tiles are smaller,
// (tx + 2)(ty + 2) <= 1300 (128 x 8 nodes at most), and the colliders load
// the reference word of their own group (the references of the populations
// in qbuf) from HBM, where the pullers read it two planes earlier: 160,224 bytes.
constexpr int SPLIT_SP_N = 1300;
template <> struct SplitLds<ST_F16N> {
    unsigned long long qbuf[3][Q][SPLIT_ROLE];
    float rbuf[3][SPLIT_NODES];
    float ring[4][SPLIT_SP_N];
    uint16_t nring[4][SPLIT_SP_N];  // binary16 densities of this step, slots as the psi ring
};

// One tile of the split step; every thread of the 512-thread block calls it.
// RING2: the tile's halo ring has more nodes than there are pulling threads,
// and the colliders take the rest (without RING2 the pullers take a ring of
// up to 2 SPLIT_ROLE nodes in two rounds; F16N always runs that way).
// NT: the populations are stored with the non-temporal cache policy.
template <int S, int OP, bool WALL, bool RING2, bool NT>
__device__ inline void tile_split(const typename Storage<S>::T *__restrict__ A, typename Storage<S>::T *__restrict__ B,
                                  const float *__restrict__ gpsi, const GridDesc &g, const Phys<float> &P, int tile,
                                  SplitLds<S> &L) {
    using R = float;
    using T = typename Storage<S>::T;
    constexpr int NPT = Lane8<S>::NPT;
    constexpr bool NREF = S == ST_F16N;
    auto &qbuf = L.qbuf;
    auto &ring = L.ring;
    const int TX = g.tx, TY = g.ty, TXG = g.tx / NPT;
    const int SX = TX + 2;
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
    // Role by wave, read as wave-uniform so the roles are scalar branches.
    const bool puller = __builtin_amdgcn_readfirstlane(threadIdx.x) < SPLIT_ROLE;
    const int rid = puller ? threadIdx.x : threadIdx.x - SPLIT_ROLE;
    // F16N: this step's rounding key, from the seed in A's tail word; the
    // first tile passes seed + 1 on in B's (nothing in this launch reads it).
    uint32_t key = 0;
    if constexpr (NREF) {
        const uint32_t seed = *reinterpret_cast<const uint32_t *>(A + (size_t)planes_of(S) * N);
        key = sr_key(seed);
        if (tile == 0 && threadIdx.x == 0)  // the whole 16-byte tail, so that saved states are deterministic
            *reinterpret_cast<uint4 *>(B + (size_t)planes_of(S) * N) = make_uint4(seed + 1, 0u, 0u, 0u);
    }

    // This thread's group (either role): nodes x0 + NPT lx .. + NPT - 1 of row
    // ly.  A group starting at nx (a ragged last tile) supplies psi of the
    // wrapped columns to the last real column.
    const int lx = rid % TXG, ly = rid / TXG;
    const bool inner = ly < TY;
    const int xa = x0 + NPT * lx;
    const bool need_in = inner && xa <= nx && ly <= ny - y0;
    const bool active = inner && xa < nx && y0 + ly < ny;
    const int gx = xa >= nx ? xa - nx : xa, gy = wrapi(y0 + (inner ? ly : 0), ny);
    const bool wl = gx == 0, wr = gx + NPT - 1 == nx - 1;
    const int cin = (ly + 1) * SX + NPT * lx + 1;
    const int nb = ly * TX + NPT * lx;  // first node slot in rbuf
    constexpr uint32_t E = sizeof(T);
    const uint32_t PB = (uint32_t)((size_t)nx * ny * E);
    PopBuf bA, bB;
    bA.set(A, N, planes_of(S));
    bB.set(B, N, planes_of(S));
    // Offsets and halo nodes are set up inside each role's branch (setup
    // below), so that neither role's loop carries the other's registers.
    NbOff8<S> oin;

    // Halo ring: nh <= (1 + CR) SPLIT_ROLE nodes.  Each puller takes node rid
    // and, without RING2 (nh <= SPLIT_ROLE), node rid + SPLIT_ROLE in a second
    // round that is never taken.  With RING2 (a ring larger than the pullers:
    // 20 nodes more for a 128-wide tile, 264 for a 256-wide FP32 one) the
    // colliders take nodes rid + SPLIT_ROLE and, for FP32, rid + 2 SPLIT_ROLE
    // after their collision, where they have time to spare.  Each form
    // measured fastest where it is used (the colliders' second round makes
    // FP32 1% faster and F16S 3% slower even where it is not taken), and
    // without RING2 the colliders' loop carries no halo code at all.
    constexpr int HR = RING2 ? 1 : 2;                // halo rounds of a puller
    constexpr int CR = NPT == 4 ? 1 : 2;             // halo rounds of a collider (RING2)
    const int nh = 2 * SX + 2 * TY;
    int chl[2], hxs[2], hys[2];
    bool halo[2];
    NbOff oh[2];
    auto setup = [&](const bool pull_role) {
    oin.set(gx, wl, wr, gy, wrapi(gy - 1, ny), wrapi(gy + 1, ny), nx);
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int h = pull_role ? rid + r * SPLIT_ROLE : rid + (r + 1) * SPLIT_ROLE;
        int hlx = -1, hly = -1;
        halo[r] = false;
        if ((pull_role ? r < HR : RING2 && r < CR) && h < nh) {
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
            halo[r] = hlx <= nx - x0 && hly <= ny - y0;
        }
        hxs[r] = wrapi(x0 + hlx, nx);
        hys[r] = wrapi(y0 + hly, ny);
        chl[r] = (hly + 1) * SX + hlx + 1;
        oh[r].set(hxs[r], wrapi(hxs[r] - 1, nx), wrapi(hxs[r] + 1, nx), hys[r], wrapi(hys[r] - 1, ny),
                  wrapi(hys[r] + 1, ny), nx, E);
    }
    };
    // Colliding waves with a halo node in the first / second round (wave-uniform).
    const bool chw = RING2 && !puller && (int)__builtin_amdgcn_readfirstlane(rid) + SPLIT_ROLE < nh;
    const bool chw2 = RING2 && CR > 1 && !puller && (int)__builtin_amdgcn_readfirstlane(rid) + 2 * SPLIT_ROLE < nh;
    auto zwrap = [&](int zp) { return WALL ? zp : wrapi(zp, nz); };
    auto rslot = [&](int z) { return ring[(z - zb + 1) & 3]; };
    auto nslot = [&](int z) -> uint16_t * {
        if constexpr (NREF) return L.nring[(z - zb + 1) & 3];
        else return nullptr;
    };
    auto bslot = [&](int z) { return (z - zb + 3) % 3; };
    // F16N: index of the group's first node in plane 0, and the nodes of a plane
    // (the source-node part of the rounding dither).
    const uint32_t nbase = (uint32_t)gy * (uint32_t)nx + (uint32_t)gx, plane_n = (uint32_t)nx * (uint32_t)ny;

    // Puller: plane p into the LDS buffers.  (Keeping the next plane's loads
    // in flight as well, or issuing the halo node's loads together with the
    // interior group's, measured slower on the tiles that fit the LDS best.)
    auto pull_plane = [&](int p) {
        R *slot = rslot(p);
        if (WALL && (p < 0 || p >= nz)) {
            const R *gp = gpsi + (p < 0 ? 0 : (size_t)nx * ny);
            if (need_in) {
#pragma unroll
                for (int k = 0; k < NPT; ++k) slot[cin + k] = gp[(size_t)gy * nx + gx + k];
            }
#pragma unroll
            for (int r = 0; r < HR; ++r)
                if (halo[r]) slot[chl[r]] = gp[(size_t)hys[r] * nx + hxs[r]];
            return;
        }
        const int pw = zwrap(p);
        Wide8 q;
        Seam8<S> sm;
        load8<S, WALL>(bA, nz, PB, pw, oin, q, sm);
        unsigned long long rw = 0;  // F16N: reference densities of the group's nodes
        if constexpr (NREF)
            rw = __builtin_bit_cast(unsigned long long,
                                    __builtin_amdgcn_raw_buffer_load_b64(
                                        bA.of(19), (int)oin.c,
                                        (int)u_so(bA, 19, __builtin_amdgcn_readfirstlane((uint32_t)pw * PB)),
                                        LBM_BUF_AUX));
        uint16_t *nsl = nslot(p);
        // The halo node's loads are consumed in the branch that issued them.
#pragma unroll
        for (int r = 0; r < HR; ++r) {
            if (halo[r]) {
                R fh[Q];
                R rh;
                if constexpr (NREF) {
                    float rth;
                    pull<S, WALL, true>(bA, nz, PB, pw, oh[r], P, fh, &rth);
                    rh = rth + sum19<R>(fh);
                    nsl[chl[r]] = nref_bits(rh);
                } else {
                    pull<S, WALL>(bA, nz, PB, pw, oh[r], P, fh);
                    rh = sum19<R>(fh);
                }
                slot[chl[r]] = pseudo_psi<R>(P, rh);
            }
        }
        fold8<S, WALL>(q, sm, nz, pw, wl, wr);
        const int bs = bslot(p);
        if (active) {
#pragma unroll
            for (int a = 0; a < Q; ++a) qbuf[bs][a][rid] = q.w[a];
        }
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            R f[Q];
            R rho;
            if constexpr (NREF) {  // deviations; the density is rt + their sum, and rbuf keeps the sum
                unpack8n(q, k, P, f);
                const R drho = sum19<R>(f);
                rho = ref_of(rw, k) + drho;
                if (need_in) nsl[cin + k] = nref_bits(rho);
                if (active) L.rbuf[bs][nb + k] = drho;
            } else {
                unpack8<S>(q, k, P, f);
                rho = sum19<R>(f);
                if (active) L.rbuf[bs][nb + k] = rho;
            }
            if (need_in) slot[cin + k] = pseudo_psi<R>(P, rho);
        }
    };
    // Collider's share of the halo ring of plane p (RING2), round r.
    auto halo_plane = [&](int p, int r) {
        R *slot = rslot(p);
        if (WALL && (p < 0 || p >= nz)) {
            const R *gp = gpsi + (p < 0 ? 0 : (size_t)nx * ny);
            if (halo[r]) slot[chl[r]] = gp[(size_t)hys[r] * nx + hxs[r]];
            return;
        }
        R fh[Q];
        R rh;
        if constexpr (NREF) {
            float rth;
            pull<S, WALL, true>(bA, nz, PB, zwrap(p), oh[r], P, fh, &rth);
            rh = rth + sum19<R>(fh);
        } else {
            pull<S, WALL>(bA, nz, PB, zwrap(p), oh[r], P, fh);
            rh = sum19<R>(fh);
        }
        const R psh = pseudo_psi<R>(P, rh);
        if (halo[r]) {
            slot[chl[r]] = psh;
            if constexpr (NREF) nslot(p)[chl[r]] = nref_bits(rh);
        }
    };
    // F16N: reference word of the group at plane c in A (the colliders'
    // copy of what the pullers read).
    auto ref_word = [&](int c) -> unsigned long long {
        return __builtin_bit_cast(unsigned long long,
                                  __builtin_amdgcn_raw_buffer_load_b64(
                                      bA.of(19), (int)oin.c,
                                      (int)u_so(bA, 19, __builtin_amdgcn_readfirstlane((uint32_t)c * PB)),
                                      LBM_BUF_AUX));
    };
    // Collider: plane c from the LDS buffers to B (rw: F16N reference word).
    auto collide_plane = [&](int c, unsigned long long rw) {
        if (!active) return;
        const int bs = bslot(c);
        Wide8 q;
#pragma unroll
        for (int a = 0; a < Q; ++a) q.w[a] = qbuf[bs][a][rid];
        const R *lo = rslot(c - 1), *mid = rslot(c), *hi = rslot(c + 1);
        // F16N: this step's references of the planes below, at and above
        // (a population leaving through a wall comes back to its own node).
        const uint16_t *nlo = nslot(c - 1), *nmid = nslot(c), *nhi = nslot(c + 1);
        const bool bot = WALL && c == 0, top = WALL && c == nz - 1;
        // The walled and orthogonal F16N kernels keep this loop rolled: one
        // node's values live at a time.  Fully unrolled they spill into the loop
        // over planes, where a spill reload also waits for the previous plane's
        // stores (the vector-memory counter counts stores too), and the walled
        // step took 1.09 ms instead of 0.83 ms on the 384 x 384 x 192 sessile
        // lattice; unrolled by two (no reload in that loop) it took 1.04 ms.  The
        // periodic non-orthogonal kernel unrolls without spilling, and rolled it
        // measured 0.57 ms instead of 0.34 ms at 256^3.
        constexpr int KU = (NREF && (WALL || OP == OP_ORTH)) ? 1 : NPT;
        std::conditional_t<KU == 1, Out8Rolled, Out8<S>> out;
        if constexpr (NREF) out.clear();
#pragma unroll KU
        for (int k = 0; k < NPT; ++k) {
            R f[Q];
            if constexpr (NREF) unpack8n(q, k, P, f);
            else unpack8<S>(q, k, P, f);
            R ax, ay, az;
            psi_stencil<R>(lo, mid, hi, cin + k, SX, ax, ay, az);
            const R mG_psi = -P.G * mid[cin + k];
            if constexpr (NREF) {
                // Deviations g from w_a rt (rt: the reference they were stored
                // against), collided in that form; a value for node x' is stored
                // as (g*_a + w_a (rt - rt'(x'))) 2^e, rt' this step's reference of
                // x' (the node itself where the value comes back from a wall),
                // rounded stochastically with the dither of this node and a.
                // The difference of two binary16 references is exact in FP32.
                const R rt = ref_of(rw, k), drho = L.rbuf[bs][nb + k];
                const R rho = rt + drho;
                const uint32_t nh = sr_node(key, (uint32_t)c * plane_n + nbase + (uint32_t)k);
                collide<R, OP, true>(f, rho, mG_psi * ax + rho * P.gx, mG_psi * ay + rho * P.gy,
                                     mG_psi * az + rho * P.gz, ax * ax + ay * ay + az * az, P, nullptr, drho, rt);
#pragma unroll
                for (int a = 0; a < Q; ++a) {
                    const bool back = (ez(a) < 0 && bot) || (ez(a) > 0 && top);
                    const uint16_t *pl = back ? nmid : (ez(a) < 0 ? nlo : (ez(a) > 0 ? nhi : nmid));
                    const int pos = back ? cin + k : cin + k + ex(a) + ey(a) * SX;
                    out.set_dithered(k, a, f16_dithered(__builtin_fmaf(P.wh(a), rt - nref_val(pl[pos]), f[a] * P.hs),
                                                        sr_dither(nh, a)));
                }
            } else {
                const R rho = L.rbuf[bs][nb + k];
                collide<R, OP>(f, rho, mG_psi * ax + rho * P.gx, mG_psi * ay + rho * P.gy, mG_psi * az + rho * P.gz,
                               ax * ax + ay * ay + az * az, P);
#pragma unroll
                for (int a = 0; a < Q; ++a) out.put(k, a, f[a], P);
            }
        }
        const uint32_t pz = __builtin_amdgcn_readfirstlane((uint32_t)c * PB);
        using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(bB.of(0), 0, 0, 0));
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, out.word(a)), bB.of(a), (int)oin.c,
                                                  (int)u_so(bB, a, pz), NT ? LBM_BUF_NT : LBM_BUF_STORE_AUX);
        }
        if constexpr (NREF) {  // the group's own references, for the next step's pull
            unsigned long long ro = 0;
#pragma unroll
            for (int k = 0; k < NPT; ++k) ro |= (unsigned long long)nmid[cin + k] << (16 * k);
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, ro), bB.of(19), (int)oin.c,
                                                  (int)u_so(bB, 19, pz), NT ? LBM_BUF_NT : LBM_BUF_STORE_AUX);
        }
    };

    // Iteration i: pullers take plane zb - 1 + i (up to ze), colliders plane
    // zb - 3 + i (from zb to ze - 1).  Every thread runs every iteration and
    // its barrier.
    // The roles run separate loops (each with its own registers live across
    // iterations) that meet at the same number of barriers.
    const int iters = (ze - zb) + 3;
    if (puller) {
        setup(true);
        for (int i = 0; i < iters; ++i) {
            const int p = zb - 1 + i;
            if (p <= ze) pull_plane(p);
            lds_barrier();
        }
    } else {
        setup(false);
        unsigned long long rw_next = 0;
        for (int i = 0; i < iters; ++i) {
            const int c = zb - 3 + i;
            // F16N: the next plane's reference word, issued a plane ahead and
            // before this plane's stores.
            const unsigned long long rw = rw_next;
            if constexpr (NREF) {
                if (c + 1 >= zb && c + 1 < ze) rw_next = ref_word(c + 1);
            }
            if (c >= zb) collide_plane(c, rw);
            if constexpr (RING2) {
                if (chw && c + 2 <= ze) halo_plane(c + 2, 0);
                if constexpr (CR > 1) {
                    if (chw2 && c + 2 <= ze) halo_plane(c + 2, 1);
                }
            }
            lds_barrier();
        }
    }
}

template <int S, int OP, bool WALL, bool RING2, bool NT>
__global__ void __launch_bounds__(2 * SPLIT_ROLE)
    k_step_split(const typename Storage<S>::T *__restrict__ A, typename Storage<S>::T *__restrict__ B,
                 const float *__restrict__ gpsi, GridDesc g, PhysD pd) {
    __shared__ SplitLds<S> lds;
    const int tile = xcd_tile(blockIdx.x, g.per_xcd);
    if (tile >= g.ntiles) return;
    Phys<float> P;
    P.load(pd);
    tile_split<S, OP, WALL, RING2, NT>(A, B, gpsi, g, P, tile, lds);
}

// ---------------------------------------------------------------------------
// Single-phase step with walls on any axis (the lid-driven cavity of
// Appendix B): no pseudopotential, one node per thread; the body force is
// rho g.  Reads through box_source, writes at the node itself.
// ---------------------------------------------------------------------------
template <int S, int OP>
__global__ void __launch_bounds__(256)
    k_single(const typename Storage<S>::T *__restrict__ A, typename Storage<S>::T *__restrict__ B, GridDesc g,
             PhysD pd) {
    using ST = Storage<S>;
    using R = typename ST::R;
    Phys<R> P;
    P.load(pd);
    const int nx = g.nx, ny = g.ny;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((long long)nx * ny));
        R f[Q];
        pull_box<S>(A, g, x, y, z, P, f);
        const R rho = sum19<R>(f);
        collide<R, OP>(f, rho, rho * P.gx, rho * P.gy, rho * P.gz, (R)0, P);
#pragma unroll
        for (int a = 0; a < Q; ++a) ST::store(B + (size_t)a * g.N + i, f[a], P.shh(a), P.hs);
    }
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

template <int S, int OP, bool PAIRS>
__global__ void LBM_STEP_ATTR
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
        if constexpr (PAIRS)
            tile_march2<S, OP, false>(src, dst, nullptr, g, P, item - rd.tile_begin, ps);
        else
            tile_march<S, OP, false>(src, dst, nullptr, g, P, item - rd.tile_begin, ps);
        lds_barrier();  // the next item reuses the LDS ring
    }
}

// Batched runs with the split step: the same work list, one 512-thread
// block per compute unit (the split step's LDS).
template <int S, int OP, bool RING2, bool NT>
__global__ void __launch_bounds__(2 * SPLIT_ROLE)
    k_batch_split(unsigned char *__restrict__ ws, const RunDesc *__restrict__ runs, int nruns, int total_tiles,
                  int parity) {
    using T = typename Storage<S>::T;
    __shared__ SplitLds<S> lds;
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
        Phys<float> P;
        P.load(rd.pd);
        const T *src = reinterpret_cast<const T *>(ws + (parity ? rd.offB : rd.offA));
        T *dst = reinterpret_cast<T *>(ws + (parity ? rd.offA : rd.offB));
        tile_split<S, OP, false, RING2, NT>(src, dst, nullptr, g, P, item - rd.tile_begin, lds);
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

// ---------------------------------------------------------------------------
// Two-pass step over z-slabs.  Pass A: psi of planes [za, zb) into a global
// psi array.  Pass B: for planes [za, zb) pull the populations again (the
// slab was just streamed by pass A and sits in the last-level cache), read
// the psi stencil from the global array, collide and store.  Every node's
// arithmetic is the same as in the fused kernel.
// ---------------------------------------------------------------------------
template <int S, bool WALL>
__global__ void __launch_bounds__(256)
    k_psi_planes(const typename Storage<S>::T *__restrict__ A, typename Storage<S>::R *__restrict__ psi, GridDesc g,
                 PhysD pd, int za, int zb) {
    using R = typename Storage<S>::R;
    Phys<R> P;
    P.load(pd);
    const long long plane = (long long)g.nx * g.ny;
    const long long n = plane * (zb - za);
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
        const int z = za + (int)(k / plane);
        const int rem = (int)(k - (long long)(z - za) * plane);
        const int x = rem % g.nx, y = rem / g.nx;
        R f[Q];
        pull_at<S, WALL>(A, g, x, y, z, P, f);
        psi[(size_t)z * plane + rem] = pseudo_psi<R>(P, sum19<R>(f));
    }
}

template <int S, int OP, bool WALL>
__global__ void __launch_bounds__(256)
    k_collide_planes(const typename Storage<S>::T *__restrict__ A, typename Storage<S>::T *__restrict__ B,
                     const typename Storage<S>::R *__restrict__ psi, const typename Storage<S>::R *__restrict__ gpsi,
                     GridDesc g, PhysD pd, int za, int zb) {
    using ST = Storage<S>;
    using R = typename ST::R;
    Phys<R> P;
    P.load(pd);
    const long long plane = (long long)g.nx * g.ny;
    const long long n = plane * (zb - za);
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
        const int z = za + (int)(k / plane);
        const int rem = (int)(k - (long long)(z - za) * plane);
        const int x = rem % g.nx, y = rem / g.nx;
        R f[Q];
        pull_at<S, WALL>(A, g, x, y, z, P, f);
        const R rho = sum19<R>(f);
        R acc[3] = {(R)0, (R)0, (R)0};
        // Same grouping as psi_stencil: axis terms, then the diagonal pairs.
        auto ps = [&](int dx, int dy, int dz) { return psi_at<R>(psi, gpsi, g, WALL, x + dx, y + dy, z + dz); };
        const R e = (R)(1.0 / 6.0), d = (R)(1.0 / 12.0);
        const R pxp = ps(1, 0, 0), pxm = ps(-1, 0, 0), pyp = ps(0, 1, 0), pym = ps(0, -1, 0);
        const R pzp = ps(0, 0, 1), pzm = ps(0, 0, -1);
        const R ppx = ps(1, 1, 0), pmm = ps(-1, -1, 0), ppm = ps(1, -1, 0), pmp = ps(-1, 1, 0);
        const R hxp = ps(1, 0, 1), hxm = ps(-1, 0, 1), hyp = ps(0, 1, 1), hym = ps(0, -1, 1);
        const R lxp = ps(1, 0, -1), lxm = ps(-1, 0, -1), lyp = ps(0, 1, -1), lym = ps(0, -1, -1);
        acc[0] = e * (pxp - pxm) + d * ((ppx - pmm) + (ppm - pmp) + (hxp - lxm) + (lxp - hxm));
        acc[1] = e * (pyp - pym) + d * ((ppx - pmm) - (ppm - pmp) + (hyp - lym) + (lyp - hym));
        acc[2] = e * (pzp - pzm) + d * ((hxp - lxm) - (lxp - hxm) + (hyp - lym) - (lyp - hym));
        const R mG_psi = -P.G * psi[(size_t)z * plane + rem];
        const R Fx = mG_psi * acc[0] + rho * P.gx;
        const R Fy = mG_psi * acc[1] + rho * P.gy;
        const R Fz = mG_psi * acc[2] + rho * P.gz;
        collide<R, OP>(f, rho, Fx, Fy, Fz, acc[0] * acc[0] + acc[1] * acc[1] + acc[2] * acc[2], P);
        PopBuf bB;
        bB.set(B, (size_t)g.N);
        const uint32_t off = (uint32_t)(((size_t)z * plane + rem) * sizeof(typename ST::T));
#pragma unroll
        for (int a = 0; a < Q; ++a) ST::stb(f[a], bB.of(a), off, bB.so(a, 0), P.shh(a), P.hs);
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
    rho_w[i] = density_at<S, true>(A, g, x, y, z, P);
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
    const int nx = g.nx, ny = g.ny;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((long long)nx * ny));
        psi[i] = pseudo_psi<R>(P, density_at<S, WALL>(A, g, x, y, z, P));
    }
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
    R rt = (R)0;  // F16N: f holds the deviations from w_a rt
    if constexpr (S == ST_F16N) rt = pull_dev_at<WALL>(A, g, x, y, z, P, f);
    else pull_at<S, WALL>(A, g, x, y, z, P, f);
    finite = true;
#pragma unroll
    for (int a = 0; a < Q; ++a) finite = finite && isfinite(f[a]);
    Pre<R> pr;
    pr.build(f);
    if constexpr (S == ST_F16N) rho = rt + pr.rho(f[0]);
    else rho = pr.rho(f[0]);
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
        if constexpr (S == ST_F16N) {  // w_a rt + h_a 2^-e, each operation rounded once in FP64
            const double rt = (double)pull_dev_at<WALL>(A, g, x, y, z, P, v);
#pragma unroll
            for (int a = 0; a < Q; ++a) f[(size_t)a * g.N + i] = mul_rounded(wclass(a), rt) + (double)v[a];
        } else {
            pull_at<S, WALL>(A, g, x, y, z, P, v);
#pragma unroll
            for (int a = 0; a < Q; ++a) f[(size_t)a * g.N + i] = (double)v[a];
        }
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
    using R = typename ST::R;
    // F16N: the node's own density, rounded to binary16, is the reference of
    // every population that arrives here; it goes to plane 19 at the node.
    NodeShift ns;
    if constexpr (S == ST_F16N) {
        const uint16_t rt = nref_bits(sum19<R>(v));
        A[(size_t)19 * g.N + ((size_t)z * g.ny + y) * g.nx + x] = rt;
        ns.set(nref_val(rt));
    }
    auto shh = [&](int a) -> R {
        if constexpr (S == ST_F16N) return ns(a) * P.hs;
        else return P.shh(a);
    };
    if (g.wall_x | g.wall_y) {
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            size_t idx;
            int d;
            bool lid;
            box_source(g, x, y, z, a, idx, d, lid);
            ST::store(A + (size_t)d * g.N + idx, lid ? v[a] - lid_term(P, a) : v[a], shh(d), P.hs);
        }
        return;
    }
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
        ST::store(A + (size_t)d * g.N + idx, v[a], shh(a), P.hs);
    }
}

// F16N from FP64 populations (periodic x and y): the reference rt is the
// node's density rounded to FP32 and then to binary16, and each value is
// (f_a - w_a rt) 2^e rounded once to binary16, the product and the
// difference taken in FP64 (each rounded once).
template <bool WALL>
__device__ inline void scatter_node_dev(uint16_t *__restrict__ A, const GridDesc &g, const Phys<float> &P, int x,
                                        int y, int z, const double f[Q]) {
    const uint16_t rb = nref_bits((float)sum19<double>(f));
    A[(size_t)19 * g.N + ((size_t)z * g.ny + y) * g.nx + x] = rb;
    const double rt = (double)nref_val(rb), hs = (double)P.hs;
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
        const _Float16 h = (_Float16)((f[a] - mul_rounded(wclass(a), rt)) * hs);
        A[(size_t)d * g.N + idx] = __builtin_bit_cast(uint16_t, h);
    }
}

// A state written from outside the step starts its rounding seed at zero.
template <int S> __device__ inline void reset_seed(typename Storage<S>::T *__restrict__ A, const GridDesc &g) {
    if constexpr (tail_elems(S) > 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0)
            *reinterpret_cast<uint4 *>(A + (size_t)planes_of(S) * g.N) = make_uint4(0u, 0u, 0u, 0u);
    }
}

template <int S, bool WALL>
__global__ void k_write_pops(typename Storage<S>::T *__restrict__ A, const double *__restrict__ f, GridDesc g,
                             PhysD pd) {
    using R = typename Storage<S>::R;
    Phys<R> P;
    P.load(pd);
    reset_seed<S>(A, g);
    const int nx = g.nx, ny = g.ny;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((long long)nx * ny));
        if constexpr (S == ST_F16N) {
            double fd[Q];
#pragma unroll
            for (int a = 0; a < Q; ++a) fd[a] = f[(size_t)a * g.N + i];
            scatter_node_dev<WALL>(A, g, P, x, y, z, fd);
        } else {
            R v[Q];
#pragma unroll
            for (int a = 0; a < Q; ++a) v[a] = (R)f[(size_t)a * g.N + i];
            scatter_node<S, WALL>(A, g, P, x, y, z, v);
        }
    }
}

template <int S, int OP, bool WALL>
__global__ void k_init_fields(typename Storage<S>::T *__restrict__ A, const double *__restrict__ rho,
                              const double *__restrict__ u, GridDesc g, PhysD pd) {
    using R = typename Storage<S>::R;
    Phys<R> P;
    P.load(pd);
    reset_seed<S>(A, g);
    const int nx = g.nx, ny = g.ny;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((long long)nx * ny));
        R v[Q];
        equilibrium<R, OP>((R)rho[i], (R)u[i], (R)u[g.N + i], (R)u[2 * g.N + i], P, v);
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
    reset_seed<S>(A, g);
    const int nx = g.nx, ny = g.ny;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((long long)nx * ny));
        double rho, u[3];
        droplet_rho_u(D, g, x, y, z, rho, u);
        R v[Q];
        equilibrium<R, OP>((R)rho, (R)u[0], (R)u[1], (R)u[2], P, v);
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

// Second pass of the diagnostics: DIAG_FINAL_THREADS threads each fold a
// fixed, strided subset of the block partials, then a tree in LDS combines
// them in a fixed order, so the result does not depend on timing.
constexpr int DIAG_FINAL_THREADS = 256;
__global__ void __launch_bounds__(DIAG_FINAL_THREADS)
    k_diag_final(const double *__restrict__ partial, int nblocks, double *__restrict__ out) {
    __shared__ double red[NDIAG][DIAG_FINAL_THREADS];
    const int t = threadIdx.x;
    double v[NDIAG];
#pragma unroll
    for (int k = 0; k < NDIAG; ++k) v[k] = 0.0;
    for (int b = t; b < nblocks; b += DIAG_FINAL_THREADS) {
#pragma unroll
        for (int k = 0; k < NDIAG; ++k) {
            const double p = partial[(size_t)b * NDIAG + k];
            v[k] = (k == 4) ? fmax(v[k], p) : v[k] + p;
        }
    }
#pragma unroll
    for (int k = 0; k < NDIAG; ++k) red[k][t] = v[k];
    __syncthreads();
    for (int stride = DIAG_FINAL_THREADS / 2; stride > 0; stride >>= 1) {
        if (t < stride) {
#pragma unroll
            for (int k = 0; k < NDIAG; ++k)
                red[k][t] = (k == 4) ? fmax(red[k][t], red[k][t + stride]) : red[k][t] + red[k][t + stride];
        }
        __syncthreads();
    }
    if (t < NDIAG) out[t] = red[t][0];
}

}  // namespace lbm
