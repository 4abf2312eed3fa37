// lbm_device.hpp -- device-side core of the double-distribution
// non-orthogonal MRT lattice Boltzmann step (Liu, He, Li & Li,
// arXiv:1510.08224): lattice constants, storage codecs, the pull of one node
// with its walls, and the collisions in the raw-moment spaces of M (Eq. 13)
// and N (Eq. 26), unrolled with the zeros of M, M^-1 (Eq. A1), N and N^-1
// (Eq. A2) removed.
//
// The temperature lattice is a template parameter NG:
//   NG = 5  the paper's D2Q5 thermal model (Sec. 2.2, Eqs. 23-30);
//   NG = 9  its D2Q9 thermal variant (Eqs. 31-33), collided with the same
//           non-orthogonal M as the flow, equilibrium of Eq. 31 with theta;
//   NG = 0  no temperature field (isothermal flow, Secs. 3.1-3.2).
//
// Layout in HBM: structure of arrays, interleaved by row.  Row y of a
// population buffer holds, one after another, row y of population 0, 1, ...,
// 9 + NG - 1 (the 9 flow populations, then the NG temperature populations),
// each `plane` elements long (the row length padded to 256 bytes), x
// fastest:
//   element (i, x, y) at y * pitch + i * plane + x,  pitch = (9 + NG) * plane.
// A node's populations then lie within one stretch of (9 + NG) row segments
// instead of in 9 + NG planes a whole lattice apart: the 28 streams a step
// reads and writes stay in a few DRAM pages (measured on MI355X: 5% more
// bandwidth for the step kernels than separate planes).
// The buffer read by a step holds, for time t, the values that streaming
// turns into the pre-collision populations at t (the post-collision values
// of t - 1 for every link that stays inside the lattice).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <type_traits>

namespace lbm {

enum Side { kLeft = 0, kRight = 1, kBottom = 2, kTop = 3 };

// D2Q9 velocities (Eq. 5, c = 1), their opposites; D2Q5 is the subset 0..4.
__host__ __device__ constexpr int ex(int i) {
    return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0);
}
__host__ __device__ constexpr int ey(int i) {
    return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0);
}
__host__ __device__ constexpr int opp(int i) {
    return i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5);
}
static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "opp");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "opp");

// D2Q9 weights (stated after Eq. 22).
__host__ __device__ constexpr double w9(int i) { return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0); }

// Lattice geometry of one solver.
struct Geom {
    int nx, ny;
    int pitch;          // elements per row of nodes (all populations)
    int px, py;         // 1 if the axis is periodic
    long long plane;    // elements from population i to i + 1 within a row
};

// Relaxation constants in one arithmetic type, rounded once on the host:
// the rates, the source factors h = 1 - s/2 of Eq. 8 (and of Eq. 24's
// operators), varpi and 1 - varpi.  The host applies the rounding a kernel
// would (double to float to nearest even, then one float operation), so the
// collisions give the results they would with the doubles converted per
// wave, without the conversions and with half the scalar registers.
template <class T>
struct Rates {
    T s3, s4, s6, s8;        // flow rates (Eq. 20)
    T h3, h4, h6, h8;        // 1 - s/2 for each of them
    T z1, z3, z4, z6, z8;    // thermal rates (Eq. 29, or Eq. 32 for D2Q9)
    T varpi, one_m_varpi;    // Eq. 28 (D2Q5) and 1 - varpi
    T theta;                 // Eq. 31 (D2Q9), 0 or 1
};

// Per-problem constants of the step (all derived on the host).
struct Coeffs {
    // D2Q9 flow rates (Eq. 20): s3 = s_e, s4 = s5 = s_nu, s6 = s7 = s_q, s8 = s_eps.
    double s3, s4, s6, s8;
    // Thermal rates.  D2Q5 (Eq. 29): z1 = z2 = zeta_alpha, z3 = zeta_e,
    // z4 = zeta_nu.  D2Q9 (Eq. 32): also z4 = z5 = zeta_nu, z6 = z7 = zeta_q,
    // z8 = zeta_eps.
    double z1, z3, z4, z6, z8;
    double varpi;       // Eq. 28 (D2Q5)
    double theta;       // Eq. 31 (D2Q9), 0 or 1
    double gbeta;       // g beta (Eq. 4)
    double ax, ay;      // external acceleration a (Eq. 4)
    double tshift;      // sum(g) + tshift = T - T0
    double toff;        // sum(g) + toff  = T  (also the stored rest temperature)
    double T0;          // reference temperature
    // Link-wise walls, per side.  Flow: a population pulled through a wall
    // in direction i is the stored opposite population plus bbf[side][i]
    // (= 6 w_i rho0 e_i . u_w).  Temperature: gsign[side] * stored opposite
    // + gconst[side][i] (anti-bounce-back: -1 and twice the even part of the
    // equilibrium at the wall, relative to the stored rest state;
    // bounce-back: +1, 0).
    double bbf[4][9];
    double gsign[4], gconst[4][9];
    // Non-equilibrium extrapolation walls (the wall passes through the
    // first/last node row or column): nee[side] = 1 for such a side,
    // tdir[side] = 1 if its temperature is Dirichlet, uw the wall velocity,
    // wT the wall temperature.  any_nee = any side.
    int nee[4], tdir[4], any_nee;
    double uw[4][2], wT[4];
    // Deviation storage scales (FP16): stored = value * scale.
    float fscale, finv, gscale, ginv;
    // FP16 storage keeps temperature populations as deviations from the rest
    // state at a reference temperature T0 + tau(x, y), linear in the node
    // position: tau = tb + tgx x + tgy y (the conduction profile between the
    // two Dirichlet walls of one axis; zero otherwise and for other
    // storage).  A population is stored relative to the reference of the
    // node that will pull it, so every pull yields deviations relative to
    // the puller's own rest state: a node subtracts gdc[i] = c_i (tgx e_x +
    // tgy e_y) from its post-collision g_i before storing it (c_i: the rest
    // weights of g^eq, Eq. 30 or 31).
    double tb, tgx, tgy;
    float gdc[9];
    // FP16 storage of a lattice periodic in x with its temperature reference
    // along y also keeps the flow populations as deviations from the
    // hydrostatic density of that reference, rho0 + r0 + rA y + rB y^2
    // (1/3 d rho / dy = a_y + g beta tau(y), Eq. 4): w_i (rho(y + e_y) -
    // rho(y)) comes off f_i before it is stored, (frA, frB: rA, rB in FP32).
    // Zero otherwise.
    double r0, rA, rB;
    float frA, frB;
    int collision;      // 0 the paper's MRT, 1 BGK, 2 orthogonal MRT (Sec. 3.2)
    // The rates above in each collision arithmetic: FP64 storage collides
    // in double, FP32 and FP16 storage in float.
    Rates<double> rd;
    Rates<float> rf;
};

template <class R> __host__ __device__ __forceinline__ const Rates<R>& rates_of(const Coeffs& C);
template <> __host__ __device__ __forceinline__ const Rates<double>& rates_of<double>(const Coeffs& C) { return C.rd; }
template <> __host__ __device__ __forceinline__ const Rates<float>& rates_of<float>(const Coeffs& C) { return C.rf; }

// Per-side constants of the NEE rebuild picked by a lane-varying side
// index, as a chain of selects.
__device__ __forceinline__ double by_side(const double (&a)[4], int s) {
    return s == 0 ? a[0] : (s == 1 ? a[1] : (s == 2 ? a[2] : a[3]));
}
__device__ __forceinline__ int by_side(const int (&a)[4], int s) {
    return s == 0 ? a[0] : (s == 1 ? a[1] : (s == 2 ? a[2] : a[3]));
}

// ---------------------------------------------------------------------------
// Storage codecs.  FP64 holds full populations; FP32 and FP16 hold
// deviations from the rest equilibrium.
// ---------------------------------------------------------------------------
template <class S> struct Codec;

template <> struct Codec<double> {
    using R = double;
    static constexpr bool kDev = false;
    __device__ static __forceinline__ double load(const double* p, float) { return *p; }
    __device__ static __forceinline__ void store(double* p, double v, float) {
        __builtin_nontemporal_store(v, p);
    }
};

template <> struct Codec<float> {
    using R = float;
    static constexpr bool kDev = true;
    __device__ static __forceinline__ float load(const float* p, float) { return *p; }
    __device__ static __forceinline__ void store(float* p, float v, float) {
        __builtin_nontemporal_store(v, p);
    }
};

template <> struct Codec<__half> {
    using R = float;
    static constexpr bool kDev = true;
    __device__ static __forceinline__ float load(const __half* p, float inv) {
        return __half2float(*p) * inv;
    }
    __device__ static __forceinline__ void store(__half* p, float v, float scale) {
        __half h = __float2half_rn(v * scale);
        __builtin_nontemporal_store(*reinterpret_cast<unsigned short*>(&h),
                                    reinterpret_cast<unsigned short*>(p));
    }
};

// Storage whose temperature deviations are taken from a position-dependent
// reference (Coeffs::tb, tgx, tgy, gdc): FP16.
template <class S>
constexpr bool kRefT = std::is_same<S, __half>::value;

// Reference temperature of node (x, y) above T0 (0 for other storage).
template <class S>
__device__ __forceinline__ double tref_at(const Coeffs& C, int x, int y) {
    if constexpr (kRefT<S>) return C.tb + C.tgx * (double)x + C.tgy * (double)y;
    else return 0.0;
}

// Reference density of node row y above rho0 (0 for other storage).
template <class S>
__device__ __forceinline__ double rref_at(const Coeffs& C, int y) {
    if constexpr (kRefT<S>) return C.r0 + C.rA * (double)y + C.rB * (double)y * (double)y;
    else return 0.0;
}

// Post-collision populations of a node in row y, in place, into the form
// they are stored in: relative to the reference of the node that pulls
// each of them (FP16: temperature by gdc; flow by the change of the
// hydrostatic reference density over the link, w_i (rho_ref(y + e_y) -
// rho_ref(y)) = w_i (rA + rB (2y + 1)) up, -w_i (rA + rB (2y - 1)) down).
template <class S, int NG, class R>
__device__ __forceinline__ void to_stored(R f[9], R g[NG > 0 ? NG : 1], const Coeffs& C, int y) {
    if constexpr (kRefT<S>) {
        const float up = C.frA + C.frB * (float)(2 * y + 1);
        const float dn = -(C.frA + C.frB * (float)(2 * y - 1));
        const float a9 = (float)(1.0 / 9.0), a36 = (float)(1.0 / 36.0);
        f[2] -= a9 * up;
        f[5] -= a36 * up;
        f[6] -= a36 * up;
        f[4] -= a9 * dn;
        f[7] -= a36 * dn;
        f[8] -= a36 * dn;
#pragma unroll
        for (int i = 1; i < NG; ++i) g[i] -= C.gdc[i];
    }
}

// ---------------------------------------------------------------------------
// Pull of one population with link-wise walls (Eqs. 9 and 25).
// The source of direction I at (x, y) is (x - e_I, y - e_I).  If that node
// lies outside a periodic axis it wraps; if it lies outside a wall the
// population is the stored opposite one at (x, y) with the wall rule.  A
// link that leaves through a top/bottom wall takes that wall's rule,
// otherwise the left/right wall's.
// ---------------------------------------------------------------------------
struct Src {
    long long off;  // element offset of the plane entry to read
    int side;       // wall side, or -1 for an interior / periodic link
};

template <int I, int PLANE0>
__device__ __forceinline__ Src source(const Geom& G, int x, int y) {
    constexpr int dx = ex(I), dy = ey(I);
    int sx = x - dx, sy = y - dy;
    int side = -1;
    if (dy != 0 && (sy < 0 || sy >= G.ny)) {
        if (G.py) sy = sy < 0 ? sy + G.ny : sy - G.ny;
        else side = sy < 0 ? kBottom : kTop;
    }
    if (dx != 0 && (sx < 0 || sx >= G.nx)) {
        if (G.px) sx = sx < 0 ? sx + G.nx : sx - G.nx;
        else if (side < 0) side = sx < 0 ? kLeft : kRight;
    }
    Src s;
    if (side < 0) {
        s.off = (long long)(PLANE0 + I) * G.plane + (long long)sy * G.pitch + sx;
    } else {
        s.off = (long long)(PLANE0 + opp(I)) * G.plane + (long long)y * G.pitch + x;
    }
    s.side = side;
    return s;
}

template <class S, int I>
__device__ __forceinline__ typename Codec<S>::R pull_f1(const S* __restrict__ src, const Geom& G, const Coeffs& C,
                                                        int x, int y) {
    using R = typename Codec<S>::R;
    const Src s = source<I, 0>(G, x, y);
    R v = Codec<S>::load(src + s.off, C.finv);
    if (s.side >= 0) v += (R)C.bbf[s.side][I];
    return v;
}

template <class S, int I>
__device__ __forceinline__ typename Codec<S>::R pull_g1(const S* __restrict__ src, const Geom& G, const Coeffs& C,
                                                        int x, int y) {
    using R = typename Codec<S>::R;
    const Src s = source<I, 9>(G, x, y);
    R v = Codec<S>::load(src + s.off, C.ginv);
    if (s.side >= 0) v = (R)C.gsign[s.side] * v + (R)C.gconst[s.side][I];
    return v;
}

// f[9] and g[NG] of node (x, y), link-wise walls and wraps resolved per link.
template <class S, int NG>
__device__ __forceinline__ void pull_node(const S* __restrict__ src, const Geom& G, const Coeffs& C, int x, int y,
                                          typename Codec<S>::R f[9], typename Codec<S>::R g[NG > 0 ? NG : 1]) {
    f[0] = Codec<S>::load(src + (long long)y * G.pitch + x, C.finv);
    f[1] = pull_f1<S, 1>(src, G, C, x, y);
    f[2] = pull_f1<S, 2>(src, G, C, x, y);
    f[3] = pull_f1<S, 3>(src, G, C, x, y);
    f[4] = pull_f1<S, 4>(src, G, C, x, y);
    f[5] = pull_f1<S, 5>(src, G, C, x, y);
    f[6] = pull_f1<S, 6>(src, G, C, x, y);
    f[7] = pull_f1<S, 7>(src, G, C, x, y);
    f[8] = pull_f1<S, 8>(src, G, C, x, y);
    if constexpr (NG > 0) {
        g[0] = Codec<S>::load(src + 9 * G.plane + (long long)y * G.pitch + x, C.ginv);
        g[1] = pull_g1<S, 1>(src, G, C, x, y);
        g[2] = pull_g1<S, 2>(src, G, C, x, y);
        g[3] = pull_g1<S, 3>(src, G, C, x, y);
        g[4] = pull_g1<S, 4>(src, G, C, x, y);
    }
    if constexpr (NG == 9) {
        g[5] = pull_g1<S, 5>(src, G, C, x, y);
        g[6] = pull_g1<S, 6>(src, G, C, x, y);
        g[7] = pull_g1<S, 7>(src, G, C, x, y);
        g[8] = pull_g1<S, 8>(src, G, C, x, y);
    }
}

// Element offset of the pull source of population PL in direction I
// relative to the node itself (uniform across a workgroup).
#define LBM_SHIFT(I, PL) ((long long)(PL) * G.plane - (long long)ey(I) * G.pitch - ex(I))

// Address p + byte_off with a 32-bit unsigned lane offset: a uniform base
// plus a 32-bit VGPR, which the hardware adds itself (global saddr form).
template <class T>
__device__ __forceinline__ T* at_bytes(T* p, unsigned byte_off) {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(p) + byte_off);
}
template <class T>
__device__ __forceinline__ const T* at_bytes(const T* p, unsigned byte_off) {
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + byte_off);
}

// Pull of one node whose every neighbour lies inside the lattice (no wall,
// no wrap).  Each plane's shift (plane offset - e_y pitch - e_x) is uniform
// across the workgroup, so it stays in scalar registers and every load adds
// the same 32-bit lane byte offset `boff` = (y * pitch + x) * sizeof(S).
template <class S, int NG>
__device__ __forceinline__ void pull_interior(const S* __restrict__ src, const Geom& G, const Coeffs& C,
                                              unsigned boff, typename Codec<S>::R f[9],
                                              typename Codec<S>::R g[NG > 0 ? NG : 1]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = Codec<S>::load(at_bytes(src + LBM_SHIFT(i, i), boff), C.finv);
#pragma unroll
    for (int i = 0; i < NG; ++i) g[i] = Codec<S>::load(at_bytes(src + LBM_SHIFT(i, 9 + i), boff), C.ginv);
}

// ---------------------------------------------------------------------------
// Buffer-resource access (one descriptor for a whole population buffer,
// per-plane offsets in scalar registers, one 32-bit lane offset shared by
// all planes).  Usable while the buffer is below 4 GiB.  Stores carry the
// cache policy CP: non-temporal (the written buffer is not read again in
// the same step, so it need not displace what is) or default (when both
// buffers fit the 256 MB last-level cache, the written buffer is read by
// the next step and is worth keeping there).
// ---------------------------------------------------------------------------
typedef unsigned int lbm_v2u __attribute__((ext_vector_type(2)));
constexpr int kCachePolicyNT = 2;
constexpr int kCachePolicyDefault = 0;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes) {
    // dword 3 = 0x00020000: 32-bit data format, the raw-buffer setting of gfx9-class GPUs
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <class S> struct Buf;
template <> struct Buf<double> {
    __device__ static __forceinline__ double load(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, float) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    }
    template <int CP>
    __device__ static __forceinline__ void store(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, double v,
                                                 float) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(lbm_v2u, v), r, vo, so, CP);
    }
};
template <> struct Buf<float> {
    __device__ static __forceinline__ float load(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, float) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
    template <int CP>
    __device__ static __forceinline__ void store(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, float v,
                                                 float) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, CP);
    }
};
template <> struct Buf<__half> {
    __device__ static __forceinline__ float load(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, float inv) {
        const unsigned short u = __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0);
        return __half2float(__ushort_as_half(u)) * inv;
    }
    template <int CP>
    __device__ static __forceinline__ void store(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so, float v,
                                                 float scale) {
        const unsigned short u = __half_as_ushort(__float2half_rn(v * scale));
        __builtin_amdgcn_raw_buffer_store_b16(u, r, vo, so, CP);
    }
};

// Interior pull through a buffer descriptor (node at y >= 1): every load is
// buffer_load voffset = the node's offset one row up, soffset = the shift of
// its population plus one row, which is never negative (the scalar offset
// is unsigned; a population moving in +x sits at least one plane in).
template <class S, int NG>
__device__ __forceinline__ void pull_interior_buf(__amdgpu_buffer_rsrc_t r, const Geom& G, const Coeffs& C,
                                                  unsigned boff, typename Codec<S>::R f[9],
                                                  typename Codec<S>::R g[NG > 0 ? NG : 1]) {
    const unsigned vb = boff - (unsigned)G.pitch * (unsigned)sizeof(S);
    if constexpr (std::is_same<S, __half>::value) {
        // Issue every 16-bit load before the first conversion: under
        // register pressure the scheduler otherwise waits for each load
        // before issuing the next.
        unsigned short u[9 + NG];
#pragma unroll
        for (int i = 0; i < 9; ++i)
            u[i] = __builtin_amdgcn_raw_buffer_load_b16(r, vb, (unsigned)((LBM_SHIFT(i, i) + G.pitch) * 2ll), 0);
#pragma unroll
        for (int i = 0; i < NG; ++i)
            u[9 + i] = __builtin_amdgcn_raw_buffer_load_b16(r, vb, (unsigned)((LBM_SHIFT(i, 9 + i) + G.pitch) * 2ll), 0);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = __half2float(__ushort_as_half(u[i])) * C.finv;
#pragma unroll
        for (int i = 0; i < NG; ++i) g[i] = __half2float(__ushort_as_half(u[9 + i])) * C.ginv;
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i)
            f[i] = Buf<S>::load(r, vb, (unsigned)((LBM_SHIFT(i, i) + G.pitch) * (long long)sizeof(S)), C.finv);
#pragma unroll
        for (int i = 0; i < NG; ++i)
            g[i] = Buf<S>::load(r, vb, (unsigned)((LBM_SHIFT(i, 9 + i) + G.pitch) * (long long)sizeof(S)), C.ginv);
    }
}

// ---------------------------------------------------------------------------
// Macroscopic values at a node (Eqs. 4, 18, 19, 27), conserved sums in FP64.
// `rho` and `Tsum` are sum(fbar) and sum(g) of the stored representation:
// full values for FP64 storage, deviations otherwise.
// ---------------------------------------------------------------------------
struct Macro {
    double rho;    // sum fbar (full: density; deviation: rho - rho0)
    double ux, uy; // velocity (rho0 = 1)
    double Tsum;   // sum g (full: T; deviation: T - T0); 0 without temperature
    double T;      // temperature (T0 without temperature)
    double Fx, Fy; // force per unit mass
};

// REF: the storage takes a reference temperature (kRefT); tau is then the
// node's reference temperature above T0 (tref_at), ignored otherwise.
template <class R, int NG, bool REF = false>
__device__ __forceinline__ Macro macro(const R f[9], const R g[NG > 0 ? NG : 1], const Coeffs& C, double tau = 0.0) {
    Macro m;
    if constexpr (NG == 0) {
        m.Tsum = 0.0;
        m.T = C.T0;
        m.Fy = C.ay;
    } else {
        double t = ((double)g[0] + (double)g[1]) + ((double)g[2] + (double)g[3]);
        if constexpr (NG == 5) {
            t += (double)g[4];
        } else {
            t += ((double)g[4] + (double)g[5]) + ((double)g[6] + (double)g[7]);
            t += (double)g[8];
        }
        m.Tsum = t;
        if constexpr (REF) {
            m.T = t + C.toff + tau;
            m.Fy = C.ay + C.gbeta * (t + C.tshift + tau);
        } else {
            m.T = t + C.toff;
            m.Fy = C.ay + C.gbeta * (t + C.tshift);
        }
    }
    m.Fx = C.ax;
    const double f0 = f[0], f1 = f[1], f2 = f[2], f3 = f[3], f4 = f[4];
    const double f5 = f[5], f6 = f[6], f7 = f[7], f8 = f[8];
    m.rho = (((f0 + f1) + (f2 + f3)) + ((f4 + f5) + (f6 + f7))) + f8;
    const double d57 = f5 - f7, d68 = f6 - f8;
    const double jx = (f1 - f3) + (d57 - d68);
    const double jy = (f2 - f4) + (d57 + d68);
    m.ux = jx + 0.5 * m.Fx;
    m.uy = jy + 0.5 * m.Fy;
    return m;
}

// macro() at node (x, y) of a lattice stored as S.
template <class S, class R, int NG>
__device__ __forceinline__ Macro macro_at(const R f[9], const R g[NG > 0 ? NG : 1], const Coeffs& C, int x, int y) {
    if constexpr (kRefT<S>) return macro<R, NG, true>(f, g, C, tref_at<S>(C, x, y));
    else return macro<R, NG>(f, g, C);
}

// a * b + c rounded once (a fused multiply-add).  The library is built
// without contraction, so every kernel that inlines an expression rounds it
// alike; the collisions name their multiply-adds explicitly.
template <class R>
__device__ __forceinline__ R fmaR(R a, R b, R c) {
    if constexpr (std::is_same<R, float>::value) return __builtin_fmaf(a, b, c);
    else return __builtin_fma(a, b, c);
}

// Relaxation of one moment toward its equilibrium with its source term
// (Eq. 8): m - s (m - m_eq) + h S.
template <class R>
__device__ __forceinline__ R relax(R m, R s, R meq, R h, R S) {
    return fmaR(h, S, fmaR(-s, m - meq, m));
}

// Rows 3..8 of the raw-moment transform M of Eq. 13 (rows 0..2 are the
// conserved sums), and its inverse (Eq. A1) from the moments k0..k8.
template <class R>
struct Moments9 {
    R m3, m4, m5, m6, m7, m8, d13, d24;
    __device__ __forceinline__ explicit Moments9(const R v[9]) {
        const R a13 = v[1] + v[3], a24 = v[2] + v[4];
        const R c57 = v[5] + v[7], c68 = v[6] + v[8];
        const R d57 = v[5] - v[7], d68 = v[6] - v[8];
        m8 = c57 + c68;
        m3 = (a13 + a24) + (R)2 * m8;
        m4 = a13 - a24;
        m5 = c57 - c68;
        m6 = d57 + d68;
        m7 = d57 - d68;
        d13 = v[1] - v[3];
        d24 = v[2] - v[4];
    }
};

template <class R>
__device__ __forceinline__ void inverse9(R v[9], R k0, R k1, R k2, R k3, R k4, R k5, R k6, R k7, R k8) {
    const R q = fmaR((R)0.25, k3, (R)(-0.5) * k8);
    const R h4 = (R)0.25 * k4;
    const R bx = (R)0.5 * (k1 - k7);
    const R by = (R)0.5 * (k2 - k6);
    v[0] = (k0 - k3) + k8;
    v[1] = (q + h4) + bx;
    v[3] = (q + h4) - bx;
    v[2] = (q - h4) + by;
    v[4] = (q - h4) - by;
    const R p86 = k8 + k6, p57 = k5 + k7;
    const R r86 = k8 - k6, r57 = k5 - k7;
    v[5] = (R)0.25 * (p86 + p57);
    v[6] = (R)0.25 * (p86 - p57);
    v[7] = (R)0.25 * (r86 + r57);
    v[8] = (R)0.25 * (r86 - r57);
}

// ---------------------------------------------------------------------------
// Collision of one node in place (Eq. 8 for fbar; Eq. 24, or its D2Q9
// counterpart, for g), given its macroscopic values.  Readings: rho0 = 1
// multiplies every velocity term of m^eq and every source moment; the
// density enters only m_0^eq, the 2/3 of m_3^eq and the 1/9 of m_8^eq;
// S~_8 = (2/3) rho0 (ux Fx + uy Fy), the moment of the Guo source (the
// printed form pairs ux with Fy).  In deviation storage the same
// expressions act on deviations: the rest state is a fixed point and every
// map here is affine in rho and T with the rest parts cancelling.
// ---------------------------------------------------------------------------
template <class R, int NG, bool FLOW_MRT = true>
__device__ __forceinline__ void collide_mrt(R f[9], R g[NG > 0 ? NG : 1], const Macro& mc, const Coeffs& C) {
    const R rho = (R)mc.rho;
    const R ux = (R)mc.ux, uy = (R)mc.uy;
    const R Fx = (R)mc.Fx, Fy = (R)mc.Fy;
    const R uyy = uy * uy, uyFy = uy * Fy;
    const R usq = fmaR(ux, ux, uyy);
    const R uF = fmaR(ux, Fx, uyFy);
    const R third = (R)(1.0 / 3.0);
    if constexpr (FLOW_MRT) {
        const Moments9<R> m(f);
        // Relaxation toward m^eq (Eq. 16) with the source of Eq. 17.
        const Rates<R>& K = rates_of<R>(C);
        const R s3 = K.s3, s4 = K.s4, s6 = K.s6, s8 = K.s8;
        const R e3 = fmaR((R)(2.0 / 3.0), rho, usq);
        const R e4 = fmaR(ux, ux, -uyy);
        const R e5 = ux * uy;
        const R e6 = third * uy;
        const R e7 = third * ux;
        const R e8 = fmaR(third, usq, (R)(1.0 / 9.0) * rho);
        const R S3 = (R)2 * uF;
        const R S4 = (R)2 * fmaR(ux, Fx, -uyFy);
        const R S5 = fmaR(ux, Fy, uy * Fx);
        const R S6 = third * Fy;
        const R S7 = third * Fx;
        const R S8 = (R)(2.0 / 3.0) * uF;
        const R n3 = relax(m.m3, s3, e3, K.h3, S3);
        const R n4 = relax(m.m4, s4, e4, K.h4, S4);
        const R n5 = relax(m.m5, s4, e5, K.h4, S5);
        const R n6 = relax(m.m6, s6, e6, K.h6, S6);
        const R n7 = relax(m.m7, s6, e7, K.h6, S7);
        const R n8 = relax(m.m8, s8, e8, K.h8, S8);
        // Conserved moments after collision: m0* = rho, m1* = jx + Fx,
        // m2* = jy + Fy (rates 1 in Eq. 20; Eq. 15 puts -F/2 in m_bar).
        const R n1 = (R)(mc.ux + 0.5 * mc.Fx);
        const R n2 = (R)(mc.uy + 0.5 * mc.Fy);
        inverse9<R>(f, rho, n1, n2, n3, n4, n5, n6, n7, n8);
    }
    if constexpr (NG == 5) {
        // n = N g (Eq. 26), n^eq (Eq. 28), Eq. 24, g* = N^-1 n* (Eq. A2).
        const R T = (R)mc.T;
        const R t0 = (R)mc.Tsum;
        const R t1 = g[1] - g[3];
        const R t2 = g[2] - g[4];
        const R t3 = (g[1] + g[3]) + (g[2] + g[4]);
        const R t4 = (g[1] + g[3]) - (g[2] + g[4]);
        const Rates<R>& K = rates_of<R>(C);
        const R z1 = K.z1, z3 = K.z3, z4 = K.z4;
        const R k1 = fmaR(-z1, fmaR(-ux, T, t1), t1);
        const R k2 = fmaR(-z1, fmaR(-uy, T, t2), t2);
        const R k3 = fmaR(-z3, fmaR(-K.varpi, t0, t3), t3);
        const R k4 = fmaR(-z4, t4, t4);
        const R w3 = (R)0.25 * k3, w4 = (R)0.25 * k4;
        const R wp = w3 + w4, wm = w3 - w4;
        g[0] = t0 - k3;
        g[1] = fmaR((R)0.5, k1, wp);
        g[3] = fmaR((R)(-0.5), k1, wp);
        g[2] = fmaR((R)0.5, k2, wm);
        g[4] = fmaR((R)(-0.5), k2, wm);
    }
    if constexpr (NG == 9) {
        // n = M g (Eq. 13), n^eq = M g^eq with g^eq of Eq. 31:
        // T (1, ux, uy, 2/3 + th |u|^2, th (ux^2 - uy^2), th ux uy, uy/3,
        // ux/3, 1/9 + th |u|^2 / 3); relaxation with Q of Eq. 32;
        // g* = M^-1 n*.  The rest part of the constant terms uses Tsum.
        const Moments9<R> m(g);
        const R T = (R)mc.T;
        const R t0 = (R)mc.Tsum;
        const Rates<R>& K = rates_of<R>(C);
        const R th = K.theta;
        const R n1 = m.d13 + m.m7;
        const R n2 = m.d24 + m.m6;
        const R z1 = K.z1, z3 = K.z3, z4 = K.z4, z6 = K.z6, z8 = K.z8;
        const R thT = th * T;
        const R k1 = fmaR(-z1, fmaR(-ux, T, n1), n1);
        const R k2 = fmaR(-z1, fmaR(-uy, T, n2), n2);
        const R k3 = fmaR(-z3, m.m3 - fmaR((R)(2.0 / 3.0), t0, thT * usq), m.m3);
        const R k4 = fmaR(-z4, fmaR(-thT, fmaR(ux, ux, -uyy), m.m4), m.m4);
        const R k5 = fmaR(-z4, fmaR(-thT, ux * uy, m.m5), m.m5);
        const R k6 = fmaR(-z6, fmaR(-third * uy, T, m.m6), m.m6);
        const R k7 = fmaR(-z6, fmaR(-third * ux, T, m.m7), m.m7);
        const R k8 = fmaR(-z8, m.m8 - fmaR((R)(1.0 / 9.0), t0, third * thT * usq), m.m8);
        inverse9<R>(g, t0, k1, k2, k3, k4, k5, k6, k7, k8);
    }
}

// ---------------------------------------------------------------------------
// The operators the paper compares its collision with (Sec. 3.2).
//
// Single relaxation time (BGK): fbar* = fbar - w (fbar - f^eq) + (1 - w/2) S
// with w = s_nu, f^eq of Eq. 22 and the Guo source in velocity space,
// S_i = w_i [3 (e_i - u).F + 9 (e_i.u)(e_i.F)]; g* = g - z (g - g^eq) with
// z = zeta_alpha and g^eq of Eq. 30 or 31.
//
// Classical MRT with an orthogonal basis (the Gram-Schmidt basis of the
// monomials 1, |e|^2, |e|^4, e_x, e_x|e|^2, e_y, e_y|e|^2, e_x^2 - e_y^2,
// e_x e_y, scaled to integer rows): moments rho, e, eps, j_x, q_x, j_y, q_y,
// p_xx, p_xy with equilibria rho, -2 rho + 3|u|^2, rho - 3|u|^2, u_x, -u_x,
// u_y, -u_y, u_x^2 - u_y^2, u_x u_y (the M_o f^eq of Eq. 22) and sources
// 0, 6 u.F, -6 u.F, F_x, -F_x, F_y, -F_y, 2 (u_x F_x - u_y F_y),
// u_x F_y + u_y F_x (M_o S); rates s_e, s_eps, s_q, s_nu; the inverse is
// M_o^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4).  The
// temperature keeps the model's own MRT.
// ---------------------------------------------------------------------------
enum Collision { kCollMRT = 0, kCollBGK = 1, kCollOrtho = 2 };

// e_i . (ax, ay) for the lattice vector e_i (components -1, 0 or 1): the
// value of ex * ax + ey * ay without its products by 0 and 1, which the
// compiler may not drop from IEEE arithmetic.
template <class R>
__device__ __forceinline__ R edot(int i, R ax, R ay) {
    const int dx = ex(i), dy = ey(i);
    if (dx == 0) return dy == 0 ? (R)0 : (dy > 0 ? ay : -ay);
    const R px = dx > 0 ? ax : -ax;
    return dy == 0 ? px : (dy > 0 ? px + ay : px - ay);
}

template <class R>
__device__ __forceinline__ void collide_flow_bgk(R f[9], const Macro& mc, const Coeffs& C) {
    const R rho = (R)mc.rho, ux = (R)mc.ux, uy = (R)mc.uy, Fx = (R)mc.Fx, Fy = (R)mc.Fy;
    const R w = rates_of<R>(C).s4, a = rates_of<R>(C).h4;
    const R usq15 = (R)1.5 * (ux * ux + uy * uy);
    const R uF3 = (R)3 * (ux * Fx + uy * Fy);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const R eu = edot<R>(i, ux, uy);
        const R eF = edot<R>(i, Fx, Fy);
        const R wi = (R)w9(i);
        const R feq = wi * (rho + (fmaR((R)4.5 * eu, eu, (R)3 * eu) - usq15));
        const R S = wi * fmaR((R)9 * eu, eF, fmaR((R)3, eF, -uF3));
        f[i] = relax(f[i], w, feq, a, S);
    }
}

template <class R>
__device__ __forceinline__ void collide_flow_ortho(R f[9], const Macro& mc, const Coeffs& C) {
    const R rho = (R)mc.rho, ux = (R)mc.ux, uy = (R)mc.uy, Fx = (R)mc.Fx, Fy = (R)mc.Fy;
    const R usq = ux * ux + uy * uy, uF = ux * Fx + uy * Fy;
    const R ax = f[1] + f[3], ay = f[2] + f[4];
    const R a = ax + ay, d = (f[5] + f[6]) + (f[7] + f[8]);
    const R d13 = f[1] - f[3], d24 = f[2] - f[4];
    const R sx = (f[5] - f[6]) - (f[7] - f[8]);   // diagonal part of j_x
    const R sy = (f[5] + f[6]) - (f[7] + f[8]);   // diagonal part of j_y
    const R m_e = ((R)-4 * f[0] - a) + (R)2 * d;
    const R m_eps = ((R)4 * f[0] - (R)2 * a) + d;
    const R m_qx = (R)-2 * d13 + sx;
    const R m_qy = (R)-2 * d24 + sy;
    const R m_xx = ax - ay;
    const R m_xy = (f[5] - f[6]) + (f[7] - f[8]);
    const Rates<R>& K = rates_of<R>(C);
    const R s_e = K.s3, s_eps = K.s8, s_q = K.s6, s_nu = K.s4;
    const R k_e = relax(m_e, s_e, fmaR((R)-2, rho, (R)3 * usq), K.h3, (R)6 * uF);
    const R k_eps = relax(m_eps, s_eps, fmaR((R)-3, usq, rho), K.h8, (R)-6 * uF);
    const R k_qx = relax(m_qx, s_q, -ux, K.h6, -Fx);
    const R k_qy = relax(m_qy, s_q, -uy, K.h6, -Fy);
    const R k_xx = relax(m_xx, s_nu, fmaR(ux, ux, -uy * uy), K.h4, (R)2 * fmaR(ux, Fx, -uy * Fy));
    const R k_xy = relax(m_xy, s_nu, ux * uy, K.h4, fmaR(ux, Fy, uy * Fx));
    // conserved moments after collision: rho, j + F (Eq. 15 puts -F/2 in j)
    const R jx = (R)(mc.ux + 0.5 * mc.Fx), jy = (R)(mc.uy + 0.5 * mc.Fy);
    // f = M_o^T D^-1 m*
    const R c0 = rho * (R)(1.0 / 9.0), c1 = k_e * (R)(1.0 / 36.0), c2 = k_eps * (R)(1.0 / 36.0);
    const R c3 = jx * (R)(1.0 / 6.0), c4 = k_qx * (R)(1.0 / 12.0);
    const R c5 = jy * (R)(1.0 / 6.0), c6 = k_qy * (R)(1.0 / 12.0);
    const R c7 = k_xx * (R)0.25, c8 = k_xy * (R)0.25;
    const R axis = (c0 - c1) - (R)2 * c2;
    const R diag = (c0 + (R)2 * c1) + c2;
    const R px = c3 - (R)2 * c4, py = c5 - (R)2 * c6;
    const R qx = c3 + c4, qy = c5 + c6;
    f[0] = (c0 - (R)4 * c1) + (R)4 * c2;
    f[1] = (axis + px) + c7;
    f[3] = (axis - px) + c7;
    f[2] = (axis + py) - c7;
    f[4] = (axis - py) - c7;
    f[5] = (diag + qx) + (qy + c8);
    f[6] = (diag - qx) + (qy - c8);
    f[7] = (diag - qx) - (qy - c8);
    f[8] = (diag + qx) - (qy + c8);
}

template <class R, int NG>
__device__ __forceinline__ void collide_thermal_bgk(R g[NG > 0 ? NG : 1], const Macro& mc, const Coeffs& C) {
    if constexpr (NG > 0) {
        const R ux = (R)mc.ux, uy = (R)mc.uy, T = (R)mc.T, t0 = (R)mc.Tsum;
        const Rates<R>& K = rates_of<R>(C);
        const R z = K.z1;
        if constexpr (NG == 5) {
            const R vp = K.varpi;
            g[0] = g[0] - z * (g[0] - K.one_m_varpi * t0);
#pragma unroll
            for (int i = 1; i < 5; ++i) {
                const R eu = edot<R>(i, ux, uy);
                g[i] = g[i] - z * (g[i] - ((R)0.25 * vp * t0 + (R)0.5 * eu * T));
            }
        } else {
            const R th = K.theta, usq15 = (R)1.5 * (ux * ux + uy * uy);
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const R eu = edot<R>(i, ux, uy);
                const R geq = (R)w9(i) * (t0 + T * ((R)3 * eu + th * ((R)4.5 * eu * eu - usq15)));
                g[i] = g[i] - z * (g[i] - geq);
            }
        }
    }
}

// Collision of one node with the operator COLL.
template <class R, int NG, int COLL>
__device__ __forceinline__ void collide(R f[9], R g[NG > 0 ? NG : 1], const Macro& mc, const Coeffs& C) {
    if constexpr (COLL == kCollBGK) {
        collide_flow_bgk<R>(f, mc, C);
        collide_thermal_bgk<R, NG>(g, mc, C);
    } else if constexpr (COLL == kCollOrtho) {
        collide_flow_ortho<R>(f, mc, C);
        collide_mrt<R, NG, false>(f, g, mc, C);
    } else {
        collide_mrt<R, NG>(f, g, mc, C);
    }
}

// ---------------------------------------------------------------------------
// Non-equilibrium extrapolation walls (the scheme the paper's Sec. 3 uses;
// reading: Guo-Zheng-Shi extrapolation of the non-equilibrium part).  A
// wall node x_b takes its pre-collision populations from its inward
// neighbour x_f:
//   fbar_i(x_b) = f_i^eq(rho(x_f), u_w) + [fbar_i(x_f) - f_i^eq(rho(x_f), u(x_f))]
//   g_i(x_b)    = g_i^eq(T_b, u_w)      + [g_i(x_f)    - g_i^eq(T(x_f), u(x_f))]
// with f^eq of Eq. 22 (rho only in the rest term, rho0 = 1 on the velocity
// terms), g^eq of Eq. 30 (D2Q5) or Eq. 31 (D2Q9), T_b the wall temperature
// (Dirichlet) or T(x_f) (adiabatic).  Corner nodes use the diagonal
// neighbour, the velocity of their top/bottom wall and a Dirichlet
// temperature if either wall has one (top/bottom first).  In deviation
// storage both equilibria are taken relative to the rest state, which
// cancels.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double feq_rep(int i, double rho, double ux, double uy) {
    const double eu = ex(i) * ux + ey(i) * uy, usq = ux * ux + uy * uy;
    return w9(i) * (rho + 1.0 * (3.0 * eu + 4.5 * eu * eu - 1.5 * usq));
}

// g^eq(T, u) minus the stored rest part g^eq(Trest, 0) (Trest = 0 for full
// values, T0 for deviations).
template <int NG>
__device__ __forceinline__ double geq_rep(int i, double T, double ux, double uy, const Coeffs& C) {
    const double eu = ex(i) * ux + ey(i) * uy;
    if constexpr (NG == 5) {
        if (i == 0) return (1.0 - C.varpi) * (T - C.toff);
        return 0.25 * C.varpi * (T - C.toff) + 0.5 * eu * T;
    } else {
        const double usq = ux * ux + uy * uy;
        return w9(i) * ((T - C.toff) + T * (3.0 * eu + C.theta * (4.5 * eu * eu - 1.5 * usq)));
    }
}

__device__ __forceinline__ bool nee_node_at(const Geom& G, const Coeffs& C, int x, int y) {
    return (C.nee[kLeft] && x == 0) || (C.nee[kRight] && x == G.nx - 1) || (C.nee[kBottom] && y == 0) ||
           (C.nee[kTop] && y == G.ny - 1);
}

// The inward neighbour of NEE wall node (x, y) and the sides it touches.
struct NeeWall {
    int fx, fy;   // inward neighbour
    int vs;       // side whose wall velocity applies
    int ts;       // side whose Dirichlet temperature applies, or -1
};

__device__ __forceinline__ NeeWall nee_wall(const Geom& G, const Coeffs& C, int x, int y) {
    const bool onL = C.nee[kLeft] && x == 0, onR = C.nee[kRight] && x == G.nx - 1;
    const bool onB = C.nee[kBottom] && y == 0, onT = C.nee[kTop] && y == G.ny - 1;
    const int sx = onL ? kLeft : (onR ? kRight : -1);
    const int sy = onB ? kBottom : (onT ? kTop : -1);
    NeeWall w;
    w.fx = x + (onL ? 1 : (onR ? -1 : 0));
    w.fy = y + (onB ? 1 : (onT ? -1 : 0));
    w.vs = sy >= 0 ? sy : sx;
    w.ts = (sy >= 0 && by_side(C.tdir, sy)) ? sy : ((sx >= 0 && by_side(C.tdir, sx)) ? sx : -1);
    return w;
}

// Rebuild of a wall node from the pre-collision populations ff, gf of its
// inward neighbour.
template <class R, int NG>
__device__ __forceinline__ void nee_rebuild(const NeeWall& w, const Coeffs& C, const R ff[9],
                                            const R gf[NG > 0 ? NG : 1], R f[9], R g[NG > 0 ? NG : 1]) {
    const Macro m = macro<R, NG>(ff, gf, C);
    const int vs = w.vs;
    const double uwx = vs == 0 ? C.uw[0][0] : (vs == 1 ? C.uw[1][0] : (vs == 2 ? C.uw[2][0] : C.uw[3][0]));
    const double uwy = vs == 0 ? C.uw[0][1] : (vs == 1 ? C.uw[1][1] : (vs == 2 ? C.uw[2][1] : C.uw[3][1]));
#pragma unroll
    for (int i = 0; i < 9; ++i)
        f[i] = (R)(feq_rep(i, m.rho, uwx, uwy) + ((double)ff[i] - feq_rep(i, m.rho, m.ux, m.uy)));
    if constexpr (NG > 0) {
        const double Tb = w.ts >= 0 ? by_side(C.wT, w.ts) : m.T;
#pragma unroll
        for (int i = 0; i < NG; ++i)
            g[i] = (R)(geq_rep<NG>(i, Tb, uwx, uwy, C) + ((double)gf[i] - geq_rep<NG>(i, m.T, m.ux, m.uy, C)));
    }
}

template <class S, int NG>
__device__ void nee_node(const S* __restrict__ src, const Geom& G, const Coeffs& C, int x, int y,
                         typename Codec<S>::R f[9], typename Codec<S>::R g[NG > 0 ? NG : 1]) {
    using R = typename Codec<S>::R;
    const NeeWall w = nee_wall(G, C, x, y);
    R ff[9], gf[NG > 0 ? NG : 1];
    pull_node<S, NG>(src, G, C, w.fx, w.fy, ff, gf);
    nee_rebuild<R, NG>(w, C, ff, gf, f, g);
}

// Pre-collision populations of any node: extrapolated on NEE walls,
// pulled everywhere else.
template <class S, int NG>
__device__ __forceinline__ void load_node(const S* __restrict__ src, const Geom& G, const Coeffs& C, int x, int y,
                                          typename Codec<S>::R f[9], typename Codec<S>::R g[NG > 0 ? NG : 1]) {
    if (C.any_nee && nee_node_at(G, C, x, y)) nee_node<S, NG>(src, G, C, x, y, f, g);
    else pull_node<S, NG>(src, G, C, x, y, f, g);
}

// Correction of the x-shifted pulls of a node in the first or last column
// after an interior pull (which read the neighbouring row's element there):
// NEE walls rebuild the node, periodic axes re-read the wrapped source,
// link-wise walls apply the wall rule to the node's own opposite
// population.
template <class S, int NG>
__device__ __forceinline__ void fix_x_edges(const S* __restrict__ src, const Geom& G, const Coeffs& C, int x, int y,
                                            typename Codec<S>::R f[9], typename Codec<S>::R g[NG > 0 ? NG : 1]) {
    using R = typename Codec<S>::R;
    if ((x == 0 && C.nee[kLeft]) || (x == G.nx - 1 && C.nee[kRight])) {
        nee_node<S, NG>(src, G, C, x, y, f, g);
        return;
    }
    auto ld = [&](int pl, int xx, int yy, float inv) -> R {
        return Codec<S>::load(src + (long long)pl * G.plane + (long long)yy * G.pitch + xx, inv);
    };
    // Populations moving in +x (1, 5, 8) at x = 0 and in -x (3, 6, 7) at
    // x = nx - 1.  The corrected values go through locals written back with
    // fixed indices (stores to different elements under different branches
    // would otherwise be merged into one indexed store, which keeps f and g
    // in scratch memory).
    R f1 = f[1], f5 = f[5], f8 = f[8], f3 = f[3], f6 = f[6], f7 = f[7];
    R g1 = 0, g5 = 0, g8 = 0, g3 = 0, g6 = 0, g7 = 0;
    if constexpr (NG > 0) {
        g1 = g[1];
        g3 = g[3];
    }
    if constexpr (NG == 9) {
        g5 = g[5];
        g8 = g[8];
        g6 = g[6];
        g7 = g[7];
    }
    if (x == 0) {
        if (G.px) {
            const int xs = G.nx - 1;
            f1 = ld(1, xs, y, C.finv);
            f5 = ld(5, xs, y - 1, C.finv);
            f8 = ld(8, xs, y + 1, C.finv);
            if constexpr (NG > 0) g1 = ld(10, xs, y, C.ginv);
            if constexpr (NG == 9) {
                g5 = ld(14, xs, y - 1, C.ginv);
                g8 = ld(17, xs, y + 1, C.ginv);
            }
        } else {
            f1 = ld(3, 0, y, C.finv) + (R)C.bbf[kLeft][1];
            f5 = ld(7, 0, y, C.finv) + (R)C.bbf[kLeft][5];
            f8 = ld(6, 0, y, C.finv) + (R)C.bbf[kLeft][8];
            if constexpr (NG > 0) g1 = (R)C.gsign[kLeft] * ld(12, 0, y, C.ginv) + (R)C.gconst[kLeft][1];
            if constexpr (NG == 9) {
                g5 = (R)C.gsign[kLeft] * ld(16, 0, y, C.ginv) + (R)C.gconst[kLeft][5];
                g8 = (R)C.gsign[kLeft] * ld(15, 0, y, C.ginv) + (R)C.gconst[kLeft][8];
            }
        }
    }
    if (x == G.nx - 1) {
        if (G.px) {
            f3 = ld(3, 0, y, C.finv);
            f6 = ld(6, 0, y - 1, C.finv);
            f7 = ld(7, 0, y + 1, C.finv);
            if constexpr (NG > 0) g3 = ld(12, 0, y, C.ginv);
            if constexpr (NG == 9) {
                g6 = ld(15, 0, y - 1, C.ginv);
                g7 = ld(16, 0, y + 1, C.ginv);
            }
        } else {
            f3 = ld(1, x, y, C.finv) + (R)C.bbf[kRight][3];
            f6 = ld(8, x, y, C.finv) + (R)C.bbf[kRight][6];
            f7 = ld(5, x, y, C.finv) + (R)C.bbf[kRight][7];
            if constexpr (NG > 0) g3 = (R)C.gsign[kRight] * ld(10, x, y, C.ginv) + (R)C.gconst[kRight][3];
            if constexpr (NG == 9) {
                g6 = (R)C.gsign[kRight] * ld(17, x, y, C.ginv) + (R)C.gconst[kRight][6];
                g7 = (R)C.gsign[kRight] * ld(14, x, y, C.ginv) + (R)C.gconst[kRight][7];
            }
        }
    }
    f[1] = f1;
    f[5] = f5;
    f[8] = f8;
    f[3] = f3;
    f[6] = f6;
    f[7] = f7;
    if constexpr (NG > 0) {
        g[1] = g1;
        g[3] = g3;
    }
    if constexpr (NG == 9) {
        g[5] = g5;
        g[8] = g8;
        g[6] = g6;
        g[7] = g7;
    }
}

}  // namespace lbm
