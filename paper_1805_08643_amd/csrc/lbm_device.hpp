// Device-side arithmetic of the D3Q19 MRT pseudopotential step for gfx950.
//
// Everything here is per-node register arithmetic: storage conversion, the
// pseudopotential, the hand-expanded forward and inverse transforms of both
// operators, and the relaxation in moment space.  The transforms are add /
// subtract networks (the matrices hold 0, +-1, +-2 and, in the inverse,
// +-1/2, +-1/4, 1/6, -1/12): no matrix cores, this step is bound by HBM.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int Q = 19;

// Velocity components in the order of Eq. (2).
__host__ __device__ constexpr int ex(int a) {
    return (a == 1 || a == 7 || a == 9 || a == 11 || a == 13) ? 1
         : (a == 2 || a == 8 || a == 10 || a == 12 || a == 14) ? -1 : 0;
}
__host__ __device__ constexpr int ey(int a) {
    return (a == 3 || a == 7 || a == 10 || a == 15 || a == 17) ? 1
         : (a == 4 || a == 8 || a == 9 || a == 16 || a == 18) ? -1 : 0;
}
__host__ __device__ constexpr int ez(int a) {
    return (a == 5 || a == 11 || a == 14 || a == 15 || a == 18) ? 1
         : (a == 6 || a == 12 || a == 13 || a == 16 || a == 17) ? -1 : 0;
}
// Eq. (2) lists each velocity next to its opposite: (1,2), (3,4), ... (17,18).
__host__ __device__ constexpr int opp(int a) { return a == 0 ? 0 : ((a & 1) ? a + 1 : a - 1); }
// Rest / axis / diagonal weights 1/3, 1/18, 1/36 (used for the F16 shift).
__host__ __device__ constexpr double wclass(int a) {
    return a == 0 ? 1.0 / 3.0 : (a <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

enum { OP_NONORTH = 0, OP_ORTH = 1 };
enum { ST_F64 = 0, ST_F32 = 1, ST_F16S = 2, ST_F16N = 3 };
// Direction planes of a population array: F16N adds a twentieth plane of
// reference densities.
__host__ __device__ constexpr int planes_of(int s) { return s == ST_F16N ? 20 : 19; }
// Storage elements after the planes of a population buffer: F16N keeps the
// seed of its stochastic rounding there (one 32-bit word, padded to 16 bytes).
__host__ __device__ constexpr int tail_elems(int s) { return s == ST_F16N ? 8 : 0; }
enum { PSI_SQRT_CS = 0, PSI_EXP = 1 };

// ---------------------------------------------------------------------------
// Physical constants in the arithmetic precision.
// ---------------------------------------------------------------------------
struct PhysD {  // host-filled, double
    double G, a, b, RT, psi0, rho0;
    double s_e, s_nu, s_q, s_pi, s_eps, s_m;
    double sigma;
    double g[3];
    double tan_wall, ghost_rho_min, rho_ref;
    int psi_form;
    int h_exp;  // F16S exponent offset: stored h = (fbar - w rho_ref) * 2^h_exp
    int visc;   // density-dependent viscosity on
    double nuV, dnu, vrhoV, vinv;
    double lid6[3];  // 6 lid_rho lid_u: moving-face term of a reflected population
    // Orthogonal operator: eps_eq = rho (w_eps + w_epsj |u|^2), pi_eq = w_xx p_eq,
    // and the share of the Eq. (16) term the eps row takes (1 or 0).
    double w_eps, w_epsj, w_xx, sig_eps;
};

__device__ inline float r_rcp(float v);
__device__ inline double r_rcp(double v);

template <class R> struct Phys {
    R G, a, b4, RT, psi0, rho0, two_over_G;
    R s_e, s_nu, s_q, s_pi, s_eps, s_m;
    R ksig_e, ksig_eps;  // 6 sigma s (times G^2 |acc|^2 gives the Eq. (16) part of c S)
    R gx, gy, gz;
    R tan_wall, ghost_rho_min;
    R shift[3];          // w_class * rho_ref
    R hs, hsi;           // 2^h_exp and 2^-h_exp (exact powers of two)
    R shs[3];            // shift * 2^h_exp
    int psi_form;
    int visc;
    R nuV, dnu, vrhoV, vinv;
    R lid6[3];
    R w_eps, w_epsj, w_epsj2, w_xx;
    R whs[3];  // class weights times 2^h_exp (exact): F16N's stored shift rt w_a 2^e is rt * whs in one rounding
    __device__ inline void load(const PhysD &d) {
        G = (R)d.G;
        a = (R)d.a;
        b4 = (R)(d.b * 0.25);
        RT = (R)d.RT;
        psi0 = (R)d.psi0;
        rho0 = (R)d.rho0;
        two_over_G = (R)(2.0 / d.G);
        s_e = (R)d.s_e;
        s_nu = (R)d.s_nu;
        s_q = (R)d.s_q;
        s_pi = (R)d.s_pi;
        s_eps = (R)d.s_eps;
        s_m = (R)d.s_m;
        // (1 - s/2) * 6 sigma |F_m|^2 / (psi^2 (1/s - 1/2)) = s * 6 sigma |F_m|^2 / psi^2
        ksig_e = (R)(6.0 * d.sigma * d.s_e * d.G * d.G);
        ksig_eps = (R)(6.0 * d.sigma * d.s_eps * d.G * d.G * d.sig_eps);
        w_eps = (R)d.w_eps;
        w_epsj = (R)d.w_epsj;
        w_epsj2 = (R)(2.0 * d.w_epsj);
        w_xx = (R)d.w_xx;
        gx = (R)d.g[0];
        gy = (R)d.g[1];
        gz = (R)d.g[2];
        tan_wall = (R)d.tan_wall;
        ghost_rho_min = (R)d.ghost_rho_min;
        shift[0] = (R)(d.rho_ref / 3.0);
        shift[1] = (R)(d.rho_ref / 18.0);
        shift[2] = (R)(d.rho_ref / 36.0);
        hs = (R)ldexp(1.0, d.h_exp);
        hsi = (R)ldexp(1.0, -d.h_exp);
        shs[0] = shift[0] * hs;
        shs[1] = shift[1] * hs;
        shs[2] = shift[2] * hs;
        whs[0] = (R)(1.0 / 3.0) * hs;
        whs[1] = (R)(1.0 / 18.0) * hs;
        whs[2] = (R)(1.0 / 36.0) * hs;
        psi_form = d.psi_form;
        visc = d.visc;
        nuV = (R)d.nuV;
        dnu = (R)d.dnu;
        vrhoV = (R)d.vrhoV;
        vinv = (R)d.vinv;
        lid6[0] = (R)d.lid6[0];
        lid6[1] = (R)d.lid6[1];
        lid6[2] = (R)d.lid6[2];
    }
    // Rate of the stress rows at a node of density rho: s_nu, or with a
    // density-dependent viscosity 1 / (3 nu + 1/2) with nu linear in rho
    // between (vrhoV, nuV) and (vrhoV + 1/vinv, nuV + dnu), clamped.
    __device__ inline R snu_at(R rho) const {
        if (!visc) return s_nu;
        R t = (rho - vrhoV) * vinv;
        t = t < (R)0 ? (R)0 : (t > (R)1 ? (R)1 : t);
        return r_rcp((R)3 * (nuV + t * dnu) + (R)0.5);
    }
    __device__ inline R sh(int a_) const { return a_ == 0 ? shift[0] : (a_ <= 6 ? shift[1] : shift[2]); }
    __device__ inline R shh(int a_) const { return a_ == 0 ? shs[0] : (a_ <= 6 ? shs[1] : shs[2]); }
    __device__ inline R wh(int a_) const { return a_ == 0 ? whs[0] : (a_ <= 6 ? whs[1] : whs[2]); }
};

// ---------------------------------------------------------------------------
// Storage traits.  T = element type in HBM, R = arithmetic type.
// ---------------------------------------------------------------------------
template <int S> struct Storage;

// Raw buffer access: descriptor over one direction plane (base, size in
// bytes), 32-bit per-lane offset, wave-uniform scalar offset.  The hardware
// range check against the plane size makes every access bounds-checked.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kBufWord3 = 0x00020000;  // dword 3 of a raw buffer descriptor on gfx9-family parts
#ifndef LBM_BUF_AUX
// Cache policy bits of the buffer accesses: 0 (default) keeps lines in L2 so
// that the halo re-reads of neighbouring tiles hit; 2 marks them
// non-temporal (measured slower on MI355X).
#define LBM_BUF_AUX 0
#endif
#ifndef LBM_BUF_STORE_AUX
// Cache policy of the buffer stores (same encoding).
#define LBM_BUF_STORE_AUX LBM_BUF_AUX
#endif
// Non-temporal policy of the split step's streaming stores, for lattices
// larger than the last-level cache: there the stores would only evict the
// lines that the next plane's reads need (measured 5-6% faster at 256^3), while
// a lattice that fits keeps its populations cached for the next step.
#define LBM_BUF_NT 2
__device__ inline rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, kBufWord3);
}

template <> struct Storage<ST_F64> {
    using T = double;
    using R = double;
    __device__ static inline R load(const T *p, R, R) { return __builtin_nontemporal_load(p); }
    __device__ static inline void store(T *p, R v, R, R) { __builtin_nontemporal_store(v, p); }
    __device__ static inline R ldb(rsrc_t r, uint32_t vo, uint32_t so, R, R) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, LBM_BUF_AUX));
    }
    __device__ static inline void stb(R v, rsrc_t r, uint32_t vo, uint32_t so, R, R) {
        using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, (int)vo, (int)so, LBM_BUF_STORE_AUX);
    }
};
template <> struct Storage<ST_F32> {
    using T = float;
    using R = float;
    __device__ static inline R load(const T *p, R, R) { return __builtin_nontemporal_load(p); }
    __device__ static inline void store(T *p, R v, R, R) { __builtin_nontemporal_store(v, p); }
    __device__ static inline R ldb(rsrc_t r, uint32_t vo, uint32_t so, R, R) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, LBM_BUF_AUX));
    }
    __device__ static inline void stb(R v, rsrc_t r, uint32_t vo, uint32_t so, R, R) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)vo, (int)so, LBM_BUF_STORE_AUX);
    }
};
// binary16 bits of h = (fbar - w rho_ref) * 2^e.  Loads return
// h 2^-e + shift; stores round v 2^e - shift 2^e, a single fused
// multiply-add whose exact result is rounded once to binary16 (the
// power-of-two factors are exact, so it is (v - shift) 2^e rounded once).
template <> struct Storage<ST_F16S> {
    using T = uint16_t;
    using R = float;
    __device__ static inline R load(const T *p, R shift, R hsi) {
        uint16_t bits = __builtin_nontemporal_load(p);
        return fmaf(__half2float(__ushort_as_half(bits)), hsi, shift);
    }
    __device__ static inline void store(T *p, R v, R shs, R hs) {
        __builtin_nontemporal_store(__half_as_ushort(__float2half_rn(fmaf(v, hs, -shs))), p);
    }
    __device__ static inline R ldb(rsrc_t r, uint32_t vo, uint32_t so, R shift, R hsi) {
        const uint16_t bits = __builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so, LBM_BUF_AUX);
        return fmaf(__half2float(__ushort_as_half(bits)), hsi, shift);
    }
    __device__ static inline void stb(R v, rsrc_t r, uint32_t vo, uint32_t so, R shs, R hs) {
        __builtin_amdgcn_raw_buffer_store_b16(__half_as_ushort(__float2half_rn(fmaf(v, hs, -shs))), r, (int)vo,
                                              (int)so, LBM_BUF_STORE_AUX);
    }
};

// binary16 relative to the pulling node: F16N stores every population that
// arrives at node x as h_a = (fbar*_a - w_a rt(x)) * 2^e in binary16, where
// rt(x) is the density of x at the step that wrote the state, itself rounded
// to binary16 and kept in plane 19 at x.  Load and store are those of F16S;
// only the shift (w_a rt(x) instead of w_a rho_ref) changes from node to node.
template <> struct Storage<ST_F16N> : Storage<ST_F16S> {};

// F16N reference density: binary16 bits of a density, and back.
__device__ inline uint16_t nref_bits(float rho) { return __half_as_ushort(__float2half_rn(rho)); }
__device__ inline float nref_val(uint16_t bits) { return __half2float(__ushort_as_half(bits)); }
// Shifts w_a rt of the three velocity classes, one FP32 product each.
struct NodeShift {
    float s[3];
    __device__ inline void set(float rt) {
        s[0] = rt * (float)(1.0 / 3.0);
        s[1] = rt * (float)(1.0 / 18.0);
        s[2] = rt * (float)(1.0 / 36.0);
    }
    __device__ inline float operator()(int a) const { return a == 0 ? s[0] : (a <= 6 ? s[1] : s[2]); }
};

// Stochastic rounding of the F16N step's stores.  Every step reads a seed
// from the source buffer's tail word and writes seed + 1 to the destination's,
// so the dither is a function of the state (deterministic, the same on graph
// replay and across the single-lattice, batched and allocation-free steps)
// and changes from step to step.  A value that the step moves by less than
// half a binary16 unit then keeps its change in expectation instead of being
// rounded back every step (stagnation), which is what makes nearest rounding
// drift in mass and density over long quasi-static runs.
//
// mix32: a 32-bit integer finaliser (xorshift-multiply rounds with the
// constants of C. Wellons' "lowbias32"); key mixes the seed once per step,
// node_hash the node index with it.
__host__ __device__ constexpr uint32_t mix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x7FEB352Du;
    h ^= h >> 15;
    h *= 0x846CA68Bu;
    h ^= h >> 16;
    return h;
}
__host__ __device__ constexpr uint32_t sr_key(uint32_t seed) { return mix32(seed + 0x9E3779B9u); }
__host__ __device__ constexpr uint32_t sr_node(uint32_t key, uint32_t node) { return mix32(node ^ key); }
// 13-bit dither of direction a at a node whose hash is nh: the top 13 bits of
// a Weyl sequence in a, so the 19 directions of a node take spread values.
__host__ __device__ constexpr uint32_t sr_dither(uint32_t nh, int a) { return (nh + (uint32_t)a * 0x9E3779B9u) >> 19; }
// x rounded stochastically to binary16: the dither added to the 13 bits that
// the conversion drops (for a result in binary16's normal range), then
// truncation toward zero, so the magnitude rounds up with probability equal
// to its fraction of a binary16 unit.
__device__ inline float f16_dithered(float x, uint32_t r) { return __uint_as_float(__float_as_uint(x) + r); }
__device__ inline _Float16 f16_stochastic(float x, uint32_t r) {
    return __builtin_bit_cast(_Float16,
                              (uint16_t)__builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(f16_dithered(x, r), 0.0f)));
}
// Two dithered values truncated to binary16 in one instruction (low half y0).
__device__ inline uint32_t f16_trunc2(float y0, float y1) {
    return __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(y0, y1));
}

// x y rounded on its own: the empty asm makes the product opaque, so that
// -ffp-contract=fast cannot fuse it into a following add (the pragma that
// would say so is not honoured under that flag).
__device__ inline double mul_rounded(double x, double y) {
    double p = x * y;
    asm volatile("" : "+v"(p));
    return p;
}

// Precision-explicit math (no silent promotion of float to double).  The
// FP32 path uses the hardware reciprocal and square root (about 1 ulp); the
// FP64 path keeps correctly rounded division and square root.
__device__ inline float r_sqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ inline double r_sqrt(double v) { return ::sqrt(v); }
__device__ inline float r_exp(float v) { return expf(v); }
__device__ inline double r_exp(double v) { return ::exp(v); }
__device__ inline float r_rcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ inline double r_rcp(double v) { return 1.0 / v; }

// Pseudopotential.  Square-root form: psi^2 = 2 (p_EOS - rho/3) / G with the
// Carnahan-Starling p_EOS = rho R T (1 + n + n^2 - n^3) / (1 - n)^3 - a rho^2,
// n = b rho / 4 (Eq. (58)).  Exponential form psi0 exp(-rho0 / rho).
template <class R> __device__ inline R pseudo_psi(const Phys<R> &P, R rho) {
    if (P.psi_form == PSI_EXP) return P.psi0 * r_exp(-P.rho0 * r_rcp(rho));
    R n = P.b4 * rho;
    R om = (R)1 - n;
    R num = (R)1 + n * ((R)1 + n * ((R)1 - n));
    R peos = rho * P.RT * num * r_rcp(om * om * om) - P.a * rho * rho;
    return r_sqrt(P.two_over_G * (peos - rho * (R)(1.0 / 3.0)));
}

// ---------------------------------------------------------------------------
// Inverse transforms, hand-expanded.  out_a = sum_k Minv[a][k] m_k.
// Non-orthogonal: the exact inverse of Eq. (12) (Appendix A with rows 13 and
// 14 taking their -1/4 in the e_x e_z column).
// ---------------------------------------------------------------------------
template <class R> __device__ inline void inv_nonorth(const R m[Q], R o[Q]) {
    const R h = (R)0.5, q4 = (R)0.25, s6 = (R)(1.0 / 6.0), t12 = (R)(1.0 / 12.0);
    // rest
    o[0] = m[0] - m[4] + m[16] + m[17] + m[18];
    // +-x
    R cx = s6 * (m[4] + m[5]) - h * (m[16] + m[17]);
    R dx = h * (m[1] - m[11] - m[13]);
    o[1] = cx + dx;
    o[2] = cx - dx;
    // +-y, +-z share the isotropic part
    R cyz = s6 * m[4] - t12 * m[5];
    R cy = cyz + q4 * m[6] - h * (m[16] + m[18]);
    R dy = h * (m[2] - m[10] - m[15]);
    o[3] = cy + dy;
    o[4] = cy - dy;
    R cz = cyz - q4 * m[6] - h * (m[17] + m[18]);
    R dz = h * (m[3] - m[12] - m[14]);
    o[5] = cz + dz;
    o[6] = cz - dz;
    // xy diagonals 7..10: (m7, m10, m11, m16)
    R a = m[16] + m[7], b = m[16] - m[7], c = m[10] + m[11], d = m[11] - m[10];
    o[7] = q4 * (a + c);
    o[8] = q4 * (a - c);
    o[9] = q4 * (b + d);
    o[10] = q4 * (b - d);
    // xz diagonals 11..14: (m8, m12, m13, m17)
    a = m[17] + m[8];
    b = m[17] - m[8];
    c = m[12] + m[13];
    d = m[13] - m[12];
    o[11] = q4 * (a + c);
    o[12] = q4 * (a - c);
    o[13] = q4 * (b + d);
    o[14] = q4 * (b - d);
    // yz diagonals 15..18: (m9, m14, m15, m18)
    a = m[18] + m[9];
    b = m[18] - m[9];
    c = m[14] + m[15];
    d = m[15] - m[14];
    o[15] = q4 * (a + c);
    o[16] = q4 * (a - c);
    o[17] = q4 * (b + d);
    o[18] = q4 * (b - d);
}

// Orthogonal (Gram-Schmidt) basis, rows in the order
// rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy, pyz, pxz,
// mx, my, mz.  Its inverse is M^T D^-1 with the squared row norms
// D = 19, 2394, 252, 10, 40, 10, 40, 10, 40, 36, 72, 12, 24, 4, 4, 4, 8, 8, 8.
template <class R> __device__ inline void inv_orth(const R m[Q], R o[Q]) {
    R r = m[0] * (R)(1.0 / 19.0);
    R e = m[1] * (R)(1.0 / 2394.0);
    R p = m[2] * (R)(1.0 / 252.0);
    R jx = m[3] * (R)0.1, qx = m[4] * (R)0.025;
    R jy = m[5] * (R)0.1, qy = m[6] * (R)0.025;
    R jz = m[7] * (R)0.1, qz = m[8] * (R)0.025;
    R pxx = m[9] * (R)(1.0 / 36.0), ixx = m[10] * (R)(1.0 / 72.0);
    R pww = m[11] * (R)(1.0 / 12.0), iww = m[12] * (R)(1.0 / 24.0);
    R pxy = m[13] * (R)0.25, pyz = m[14] * (R)0.25, pxz = m[15] * (R)0.25;
    R mx = m[16] * (R)0.125, my = m[17] * (R)0.125, mz = m[18] * (R)0.125;

    o[0] = r - (R)30 * e + (R)12 * p;
    R ax = r - (R)11 * e - (R)4 * p;  // common to the six axis velocities
    R x1 = ax + (R)2 * pxx - (R)4 * ixx;
    R x2 = jx - (R)4 * qx;
    o[1] = x1 + x2;
    o[2] = x1 - x2;
    R y1 = ax - pxx + (R)2 * ixx + pww - (R)2 * iww;
    R y2 = jy - (R)4 * qy;
    o[3] = y1 + y2;
    o[4] = y1 - y2;
    R z1 = ax - pxx + (R)2 * ixx - pww + (R)2 * iww;
    R z2 = jz - (R)4 * qz;
    o[5] = z1 + z2;
    o[6] = z1 - z2;
    R dg = r + (R)8 * e + p;  // common to the twelve diagonals
    R sx = jx + qx, sy = jy + qy, sz = jz + qz;
    // xy plane
    R cxy = dg + pxx + ixx + pww + iww;
    o[7] = cxy + sx + sy + pxy + mx - my;
    o[8] = cxy - sx - sy + pxy - mx + my;
    o[9] = cxy + sx - sy - pxy + mx + my;
    o[10] = cxy - sx + sy - pxy - mx - my;
    // xz plane
    R cxz = dg + pxx + ixx - pww - iww;
    o[11] = cxz + sx + sz + pxz - mx + mz;
    o[12] = cxz - sx - sz + pxz + mx - mz;
    o[13] = cxz + sx - sz - pxz - mx - mz;
    o[14] = cxz - sx + sz - pxz + mx + mz;
    // yz plane
    R cyz = dg - (R)2 * pxx - (R)2 * ixx;
    o[15] = cyz + sy + sz + pyz + my - mz;
    o[16] = cyz - sy - sz + pyz - my + mz;
    o[17] = cyz + sy - sz - pyz + my + mz;
    o[18] = cyz - sy + sz - pyz - my - mz;
}

// Partial sums shared by both forward transforms.
template <class R> struct Pre {
    R a12, a34, a56;   // axis pair sums
    R d12, d34, d56;   // axis pair differences
    R s16, s17, s18;   // sums of the xy, xz, yz diagonal quartets
    R p7, p8, p9;      // (f7+f8)-(f9+f10), (f11+f12)-(f13+f14), (f15+f16)-(f17+f18)
    R c10, c11, c12, c13, c14, c15;  // e_x^2 e_y, e_x e_y^2, e_x^2 e_z, e_x e_z^2, e_y^2 e_z, e_y e_z^2
    __device__ inline void build(const R f[Q]) {
        a12 = f[1] + f[2];
        a34 = f[3] + f[4];
        a56 = f[5] + f[6];
        d12 = f[1] - f[2];
        d34 = f[3] - f[4];
        d56 = f[5] - f[6];
        R u78 = f[7] + f[8], u910 = f[9] + f[10], v78 = f[7] - f[8], v910 = f[9] - f[10];
        R u1112 = f[11] + f[12], u1314 = f[13] + f[14], v1112 = f[11] - f[12], v1314 = f[13] - f[14];
        R u1516 = f[15] + f[16], u1718 = f[17] + f[18], v1516 = f[15] - f[16], v1718 = f[17] - f[18];
        s16 = u78 + u910;
        s17 = u1112 + u1314;
        s18 = u1516 + u1718;
        p7 = u78 - u910;
        p8 = u1112 - u1314;
        p9 = u1516 - u1718;
        c10 = v78 - v910;
        c11 = v78 + v910;
        c12 = v1112 - v1314;
        c13 = v1112 + v1314;
        c14 = v1516 - v1718;
        c15 = v1516 + v1718;
    }
    __device__ inline R rho(R f0) const { return f0 + a12 + a34 + a56 + s16 + s17 + s18; }
    __device__ inline R jx() const { return d12 + c11 + c13; }
    __device__ inline R jy() const { return d34 + c10 + c15; }
    __device__ inline R jz() const { return d56 + c12 + c14; }
};

// ---------------------------------------------------------------------------
// Collision at one node, in place on f (the pulled fbar(x, t)):
//   fbar* = fbar + Minv (m* - m),
// which equals Minv m* because Minv M = I.  m* - m is zero for rho, F for the
// momentum rows (independent of their rate: rho u = j + F/2), and
// s_k (m_eq,k - m_k) + (1 - s_k/2) S_k otherwise (Eq. (4)).
// acc = sum_a w_a psi(x + e_a) e_a, so F_m = -G psi acc and
// |F_m|^2 / psi^2 = G^2 |acc|^2 (no division by psi).
//
// DEV: f holds the deviations g_a = fbar_a - w_a rt from the rest state of a
// reference density rt, with drho = sum_a g_a and rho = rt + drho.  The rest
// state's moments are known exactly (rt for the density and energy rows, rt/9
// for the three fourth-order rows, -11 rt and 3 rt for the orthogonal e and
// eps rows, zero elsewhere), so the rows that hold them take their differences
// from drho instead of subtracting two numbers of the size of rho; the other
// rows are unchanged, and the update g* = g + Minv (m* - m) keeps the form.
// ---------------------------------------------------------------------------
template <class R, int OP, bool DEV = false>
__device__ inline void collide(R f[Q], R rho, R Fx, R Fy, R Fz, R acc2, const Phys<R> &P,
                               R *uout = nullptr, R drho = (R)0, R rt = (R)0) {
    Pre<R> pr;
    pr.build(f);
    const R inv_rho = r_rcp(rho);
    const R ux = (pr.jx() + (R)0.5 * Fx) * inv_rho;
    const R uy = (pr.jy() + (R)0.5 * Fy) * inv_rho;
    const R uz = (pr.jz() + (R)0.5 * Fz) * inv_rho;
    if (uout) {
        uout[0] = ux;
        uout[1] = uy;
        uout[2] = uz;
    }
    const R uxx = ux * ux, uyy = uy * uy, uzz = uz * uz, u2 = uxx + uyy + uzz;
    const R Fux = Fx * ux, Fuy = Fy * uy, Fuz = Fz * uz, Fu = Fux + Fuy + Fuz;
    const R third = (R)(1.0 / 3.0);
    R dm[Q];
    dm[0] = (R)0;
    dm[1] = Fx;
    dm[2] = Fy;
    dm[3] = Fz;
    const R snu = P.snu_at(rho);
    if (OP == OP_NONORTH) {
        const R ce = (R)1 - (R)0.5 * P.s_e, cn = (R)1 - (R)0.5 * snu;
        const R cq = (R)1 - (R)0.5 * P.s_q, cp = (R)1 - (R)0.5 * P.s_pi;
        // second order, Eqs. (8), (13), (14), (16)
        R m4 = pr.a12 + pr.a34 + pr.a56 + (R)2 * (pr.s16 + pr.s17 + pr.s18);
        R m5 = (R)2 * pr.a12 - pr.a34 - pr.a56 + pr.s16 + pr.s17 - (R)2 * pr.s18;
        R m6 = pr.a34 - pr.a56 + pr.s16 - pr.s17;
        dm[4] = P.s_e * ((DEV ? drho : rho) + rho * u2 - m4) + ce * (R)2 * Fu + P.ksig_e * acc2;
        dm[5] = snu * (rho * ((R)2 * uxx - uyy - uzz) - m5) + cn * (R)2 * ((R)2 * Fux - Fuy - Fuz);
        dm[6] = snu * (rho * (uyy - uzz) - m6) + cn * (R)2 * (Fuy - Fuz);
        dm[7] = snu * (rho * ux * uy - pr.p7) + cn * (Fx * uy + Fy * ux);
        dm[8] = snu * (rho * ux * uz - pr.p8) + cn * (Fx * uz + Fz * ux);
        dm[9] = snu * (rho * uy * uz - pr.p9) + cn * (Fy * uz + Fz * uy);
        // third order, Eq. (9)
        const R rx = third * rho * ux, ry = third * rho * uy, rz = third * rho * uz;
        const R qx = cq * third * Fx, qy = cq * third * Fy, qz = cq * third * Fz;
        dm[10] = P.s_q * (ry - pr.c10) + qy;
        dm[11] = P.s_q * (rx - pr.c11) + qx;
        dm[12] = P.s_q * (rz - pr.c12) + qz;
        dm[13] = P.s_q * (rx - pr.c13) + qx;
        dm[14] = P.s_q * (rz - pr.c14) + qz;
        dm[15] = P.s_q * (ry - pr.c15) + qy;
        // fourth order, Eq. (10)
        const R phi = DEV ? (R)(1.0 / 9.0) * (drho - (R)1.5 * rho * u2) : rho * (R)(1.0 / 9.0) * ((R)1 - (R)1.5 * u2);
        const R k2 = cp * (R)2 * third;
        dm[16] = P.s_pi * (phi + third * rho * (uxx + uyy) - pr.s16) + k2 * (Fux + Fuy);
        dm[17] = P.s_pi * (phi + third * rho * (uxx + uzz) - pr.s17) + k2 * (Fux + Fuz);
        dm[18] = P.s_pi * (phi + third * rho * (uyy + uzz) - pr.s18) + k2 * (Fuy + Fuz);
        R o[Q];
        inv_nonorth<R>(dm, o);
#pragma unroll
        for (int a = 0; a < Q; ++a) f[a] += o[a];
    } else {
        // Orthogonal model: m_eq = M_orth f_eq (textbook D3Q19 equilibrium),
        // S = M_orth G (Guo forcing), or with eps_eq and pi_eq from the
        // parameters (w_eps, w_epsj, w_xx) and their source rows; Eq. (16)
        // term carried to the e and eps rows by the image of the
        // non-orthogonal column (19, -16), or to e only.
        const R ce = (R)1 - (R)0.5 * P.s_e, cE = (R)1 - (R)0.5 * P.s_eps;
        const R cn = (R)1 - (R)0.5 * snu, cq = (R)1 - (R)0.5 * P.s_q;
        const R cp = (R)1 - (R)0.5 * P.s_pi;
        const R sumax = pr.a12 + pr.a34 + pr.a56, sumdg = pr.s16 + pr.s17 + pr.s18;
        const R e = (R)(-30) * f[0] - (R)11 * sumax + (R)8 * sumdg;
        const R eps = (R)12 * f[0] - (R)4 * sumax + sumdg;
        const R qxm = (R)(-4) * pr.d12 + pr.c11 + pr.c13;
        const R qym = (R)(-4) * pr.d34 + pr.c10 + pr.c15;
        const R qzm = (R)(-4) * pr.d56 + pr.c12 + pr.c14;
        const R pxx = (R)2 * pr.a12 - pr.a34 - pr.a56 + pr.s16 + pr.s17 - (R)2 * pr.s18;
        const R ixx = (R)(-4) * pr.a12 + (R)2 * (pr.a34 + pr.a56) + pr.s16 + pr.s17 - (R)2 * pr.s18;
        const R pww = pr.a34 - pr.a56 + pr.s16 - pr.s17;
        const R iww = (R)(-2) * (pr.a34 - pr.a56) + pr.s16 - pr.s17;
        const R mx = pr.c11 - pr.c13, my = pr.c15 - pr.c10, mz = pr.c12 - pr.c14;
        const R dxx = (R)2 * uxx - uyy - uzz, dww = uyy - uzz;
        const R Sxx = (R)2 * ((R)2 * Fux - Fuy - Fuz), Sww = (R)2 * (Fuy - Fuz);
        const R two3 = (R)(2.0 / 3.0);
        dm[0] = (R)0;
        const R e_eq = DEV ? (R)(-11) * drho + (R)19 * rho * u2 : rho * ((R)(-11) + (R)19 * u2);
        const R eps_eq = DEV ? P.w_eps * drho + (P.w_eps - (R)3) * rt + P.w_epsj * rho * u2
                             : rho * (P.w_eps + P.w_epsj * u2);
        dm[1] = P.s_e * (e_eq - e) + ce * (R)38 * Fu + (R)19 * P.ksig_e * acc2;
        dm[2] = P.s_eps * (eps_eq - eps) + cE * P.w_epsj2 * Fu - (R)16 * P.ksig_eps * acc2;
        dm[3] = Fx;
        dm[4] = P.s_q * (-two3 * rho * ux - qxm) - cq * two3 * Fx;
        dm[5] = Fy;
        dm[6] = P.s_q * (-two3 * rho * uy - qym) - cq * two3 * Fy;
        dm[7] = Fz;
        dm[8] = P.s_q * (-two3 * rho * uz - qzm) - cq * two3 * Fz;
        dm[9] = snu * (rho * dxx - pxx) + cn * Sxx;
        dm[10] = P.s_pi * (P.w_xx * rho * dxx - ixx) + cp * P.w_xx * Sxx;
        dm[11] = snu * (rho * dww - pww) + cn * Sww;
        dm[12] = P.s_pi * (P.w_xx * rho * dww - iww) + cp * P.w_xx * Sww;
        dm[13] = snu * (rho * ux * uy - pr.p7) + cn * (Fx * uy + Fy * ux);
        dm[14] = snu * (rho * uy * uz - pr.p9) + cn * (Fy * uz + Fz * uy);
        dm[15] = snu * (rho * ux * uz - pr.p8) + cn * (Fx * uz + Fz * ux);
        dm[16] = -P.s_m * mx;
        dm[17] = -P.s_m * my;
        dm[18] = -P.s_m * mz;
        R o[Q];
        inv_orth<R>(dm, o);
#pragma unroll
        for (int a = 0; a < Q; ++a) f[a] += o[a];
    }
}

// Equilibrium populations M^-1 m_eq(rho, u) of either operator.
template <class R, int OP>
__device__ inline void equilibrium(R rho, R ux, R uy, R uz, const Phys<R> &P, R f[Q]) {
    const R uxx = ux * ux, uyy = uy * uy, uzz = uz * uz, u2 = uxx + uyy + uzz;
    const R third = (R)(1.0 / 3.0);
    R m[Q];
    if (OP == OP_NONORTH) {
        m[0] = rho;
        m[1] = rho * ux;
        m[2] = rho * uy;
        m[3] = rho * uz;
        m[4] = rho + rho * u2;
        m[5] = rho * ((R)2 * uxx - uyy - uzz);
        m[6] = rho * (uyy - uzz);
        m[7] = rho * ux * uy;
        m[8] = rho * ux * uz;
        m[9] = rho * uy * uz;
        m[10] = third * rho * uy;
        m[11] = third * rho * ux;
        m[12] = third * rho * uz;
        m[13] = third * rho * ux;
        m[14] = third * rho * uz;
        m[15] = third * rho * uy;
        const R phi = rho * (R)(1.0 / 9.0) * ((R)1 - (R)1.5 * u2);
        m[16] = phi + third * rho * (uxx + uyy);
        m[17] = phi + third * rho * (uxx + uzz);
        m[18] = phi + third * rho * (uyy + uzz);
        inv_nonorth<R>(m, f);
    } else {
        const R two3 = (R)(2.0 / 3.0);
        const R dxx = (R)2 * uxx - uyy - uzz, dww = uyy - uzz;
        m[0] = rho;
        m[1] = rho * ((R)(-11) + (R)19 * u2);
        m[2] = rho * (P.w_eps + P.w_epsj * u2);
        m[3] = rho * ux;
        m[4] = -two3 * rho * ux;
        m[5] = rho * uy;
        m[6] = -two3 * rho * uy;
        m[7] = rho * uz;
        m[8] = -two3 * rho * uz;
        m[9] = rho * dxx;
        m[10] = P.w_xx * rho * dxx;
        m[11] = rho * dww;
        m[12] = P.w_xx * rho * dww;
        m[13] = rho * ux * uy;
        m[14] = rho * uy * uz;
        m[15] = rho * ux * uz;
        m[16] = m[17] = m[18] = (R)0;
        inv_orth<R>(m, f);
    }
}

}  // namespace lbm
