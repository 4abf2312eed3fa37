// lbm_kernels.hip -- gfx950 kernels of the non-orthogonal MRT lattice
// Boltzmann step and its readouts, for every temperature lattice NG (0, 5, 9)
// and storage (FP64, FP32 / FP16 deviations).
//
//   k_sweep          fused pull-stream + walls + Boussinesq force + flow and
//                    temperature collision + store (one time step; Eqs. 4, 8,
//                    9, 24, 25)
//   k_sweep_batch    the same step for every lattice of a batch
//   k_sweep2(_batch) two time steps per launch: the first on a tile and its
//                    halo into LDS, the second from LDS to memory
//   k_sweepk(_batch) K time steps per launch (FP64 / FP32, D2Q5 or no
//                    temperature: four; FP64 D2Q9 thermal: three): the tile
//                    grown by K - 1 nodes from memory into LDS, grown by
//                    K - 2 .. 1 within LDS, the tile to memory
//   k_moments        rho, u, T at time t (Eqs. 18, 19, 27)
//   k_gather         pre-collision populations at time t, FP64
//   k_unstream       write a buffer whose pull yields given pre-collision
//                    populations (state restore and initial equilibrium)
//   k_nusselt_local  local wall Nusselt numbers (Eq. 39 and the local
//                    definition before it), one thread per wall node
//   k_nusselt_reduce their mean and maximum, one block, fixed-order FP64
//   k_residual(_batch) steady-state residual and non-finite count, FP64,
//                    reduced in a fixed order by k_reduce_final / k_reduce_members
//
// All kernels read the state through load_node / pull_node / source
// (lbm_device.hpp), so the wall rules exist in one place.
#include "lbm_internal.hpp"

#include <float.h>
#include <type_traits>
#include <utility>
#include <math.h>

namespace lbm {

constexpr int gdim(int NG) { return NG > 0 ? NG : 1; }

// Workgroup b runs on XCD b % 8 of the MI355X; each XCD has its own L2.
// Tile orders (tiles numbered row-major, tiles_x per row):
//   kXcdRoundRobin  tile b: with a multiple of 8 tiles per row, XCD k takes
//                   the tile columns k, k + 8, ...; neighbouring tiles of a
//                   row sit on different XCDs, so the cache lines that their
//                   x-shifted pulls share are fetched twice;
//   kXcdBands       each XCD takes a contiguous range of tiles (a band of
//                   rows): shared lines stay in one L2;
//   kXcdStrips      each XCD takes a contiguous eighth of every row (needs
//                   a multiple of 8 tiles per row): shared lines stay in one
//                   L2 except at the 8 strip edges, and all XCDs stream
//                   through the same rows together.
// Which is fastest depends on how much of the state the caches hold; the
// host picks.
enum XcdOrder { kXcdRoundRobin = 0, kXcdBands = 1, kXcdStrips = 2 };

__device__ __forceinline__ int xcd_remap(int b, int n, int order, int tiles_x) {
    if (order == kXcdRoundRobin) return b;
    const int xcd = b & 7, idx = b >> 3;
    if (order == kXcdStrips) {
        const int w = tiles_x >> 3;
        return (idx / w) * tiles_x + xcd * w + idx % w;
    }
    const int q = n >> 3, r = n & 7;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// Bytes of one population buffer: ny rows of pitch elements.
template <class S>
static unsigned long long buffer_bytes(const Geom& G) {
    return (unsigned long long)G.ny * (unsigned long long)G.pitch * sizeof(S);
}

template <class S, int NG>
__device__ __forceinline__ void store_node(S* __restrict__ dst, const Geom& G, const Coeffs& C, unsigned boff,
                                           const typename Codec<S>::R f[9],
                                           const typename Codec<S>::R g[gdim(NG)]) {
#pragma unroll
    for (int i = 0; i < 9; ++i) Codec<S>::store(at_bytes(dst + (long long)i * G.plane, boff), f[i], C.fscale);
#pragma unroll
    for (int i = 0; i < NG; ++i)
        Codec<S>::store(at_bytes(dst + (long long)(9 + i) * G.plane, boff), g[i], C.gscale);
}

template <class S, int NG, int CP>
__device__ __forceinline__ void store_node_buf(__amdgpu_buffer_rsrc_t r, const Geom& G, const Coeffs& C,
                                               unsigned boff, const typename Codec<S>::R f[9],
                                               const typename Codec<S>::R g[gdim(NG)]) {
#pragma unroll
    for (int i = 0; i < 9; ++i)
        Buf<S>::template store<CP>(r, boff, (unsigned)((long long)i * G.plane * (long long)sizeof(S)), f[i],
                                   C.fscale);
#pragma unroll
    for (int i = 0; i < NG; ++i)
        Buf<S>::template store<CP>(r, boff, (unsigned)((long long)(9 + i) * G.plane * (long long)sizeof(S)), g[i],
                                   C.gscale);
}

// Addressing and store modes of the step kernels.
enum Mode {
    kGlobal = 0,     // 64-bit addresses, non-temporal stores (buffers of 4 GiB or more)
    kBufferNT = 1,   // buffer descriptors, non-temporal stores
    kBufferKeep = 2  // buffer descriptors, default-policy stores (state fits the last-level cache)
};

// One time step of the nodes (x, y0 .. y0 + ROWS - 1) of one lattice.
// Fast path (wave-uniform): a wave whose 64 columns all lie in the lattice
// and whose rows all have a row above and below reads every population
// with one shared lane offset, all ROWS x (9 + NG) loads issued before any
// arithmetic; lanes in the first or last column then correct their
// x-shifted pulls.  Waves touching the bottom or top row, or the ragged
// right end, resolve walls and wraps per link.  MODE selects the addressing
// and the store policy of the fast path, COLL the collision operator.
template <class S, int NG, int ROWS, int MODE, int COLL>
__device__ __forceinline__ void sweep_nodes(const Geom& G, const Coeffs& C, const S* __restrict__ src,
                                            S* __restrict__ dst, int x, int y0, unsigned buf_bytes) {
    using R = typename Codec<S>::R;
    const int xw = __builtin_amdgcn_readfirstlane(x);
    const int yw = __builtin_amdgcn_readfirstlane(y0);
    const bool fast = xw + 63 <= G.nx - 1 && yw >= 1 && yw + ROWS - 1 <= G.ny - 2;
    if (fast) {
        R f[ROWS][9], g[ROWS][gdim(NG)];
        // buffer modes: byte offset of the node in its buffer (below 4 GiB);
        // 64-bit addresses: the row's offset goes into the pointer, the
        // lane offset is the node's byte offset within the row
        unsigned boff[ROWS];
#pragma unroll
        for (int r = 0; r < ROWS; ++r)
            boff[r] = MODE != kGlobal ? (unsigned)((y0 + r) * G.pitch + x) * (unsigned)sizeof(S)
                                      : (unsigned)x * (unsigned)sizeof(S);
        if (MODE != kGlobal) {
            const __amdgpu_buffer_rsrc_t rs = make_rsrc(src, buf_bytes);
#pragma unroll
            for (int r = 0; r < ROWS; ++r) pull_interior_buf<S, NG>(rs, G, C, boff[r], f[r], g[r]);
        } else {
#pragma unroll
            for (int r = 0; r < ROWS; ++r)
                pull_interior<S, NG>(src + (long long)(y0 + r) * G.pitch, G, C, boff[r], f[r], g[r]);
        }
        if (xw == 0 || xw + 63 == G.nx - 1) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) fix_x_edges<S, NG>(src, G, C, x, y0 + r, f[r], g[r]);
        }
#pragma unroll
        for (int r = 0; r < ROWS; ++r) {
            const Macro m = macro_at<S, R, NG>(f[r], g[r], C, x, y0 + r);
            collide<R, NG, COLL>(f[r], g[r], m, C);
            to_stored<S, NG>(f[r], g[r], C, y0 + r);
            if (MODE == kBufferNT)
                store_node_buf<S, NG, kCachePolicyNT>(make_rsrc(dst, buf_bytes), G, C, boff[r], f[r], g[r]);
            else if (MODE == kBufferKeep)
                store_node_buf<S, NG, kCachePolicyDefault>(make_rsrc(dst, buf_bytes), G, C, boff[r], f[r], g[r]);
            else
                store_node<S, NG>(dst + (long long)(y0 + r) * G.pitch, G, C, boff[r], f[r], g[r]);
        }
        return;
    }
    if (x >= G.nx) return;
    R f[ROWS][9], g[ROWS][gdim(NG)];
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
        if (y0 + r < G.ny) load_node<S, NG>(src, G, C, x, y0 + r, f[r], g[r]);
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        if (y0 + r < G.ny) {
            const Macro m = macro_at<S, R, NG>(f[r], g[r], C, x, y0 + r);
            collide<R, NG, COLL>(f[r], g[r], m, C);
            to_stored<S, NG>(f[r], g[r], C, y0 + r);
            store_node<S, NG>(dst + (long long)(y0 + r) * G.pitch, G, C, (unsigned)x * (unsigned)sizeof(S), f[r],
                              g[r]);
        }
    }
}

// One time step of one lattice: tiles of blockDim.x x (blockDim.y * ROWS)
// nodes, in the XCD order `remap`.
// The step constants come by pointer to device memory: a lane-varying
// index into them (the wall tables) is then a plain load, where an index
// into a by-value kernel argument would make the compiler copy the whole
// argument to scratch memory in every lane.
template <class S, int NG, int ROWS, int MODE, int COLL>
__global__ __launch_bounds__(256) void k_sweep(Geom G, const Coeffs* __restrict__ Cp, const S* __restrict__ src,
                                               S* __restrict__ dst, int tiles_x, unsigned buf_bytes, int remap) {
    const Coeffs& C = *Cp;
    const int tile = xcd_remap(blockIdx.x, gridDim.x, remap, tiles_x);
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int x = tx * blockDim.x + threadIdx.x;
    const int y0 = (ty * blockDim.y + threadIdx.y) * ROWS;
    sweep_nodes<S, NG, ROWS, MODE, COLL>(G, C, src, dst, x, y0, buf_bytes);
}

// ---------------------------------------------------------------------------
// Two time steps per launch.  A workgroup owns a tile of 64 x TY nodes.
// First it runs the step t -> t + 1 on the tile and a one-node halo around
// it, reading the state from HBM as the single-step kernel does, and keeps
// in LDS the post-collision populations that the tile pulls next (rounded
// exactly as a store to the storage type would round them).  Then it runs
// the step t + 1 -> t + 2 on the tile, pulling from LDS, and stores to HBM.
// Every population crosses HBM once per two steps instead of once per
// step; the halo costs (66 (TY + 2)) / (64 TY) - 1 extra collisions.  The
// result is bitwise the result of two single steps.
//
// LDS layout: population i of the second step's pull at tile node n comes
// from node n - e_i.  In the halo layout plane i covers the whole slot grid
// of the first step (66 x (TY + 2)): every slot stores all its populations
// at its own index, without a test and from one address with constant
// offsets, and the second step reads slot n - e_i, again one address with
// constant offsets.  In the window layout (FP64 D2Q9 thermal, whose halo
// planes would take more than half a CU's LDS) plane i holds exactly the 64 x TY
// window the tile pulls (the tile shifted by -e_i), indexed by the pulling
// node, and a first-step node writes population i to n + e_i when that
// lies in the tile.  Where the link into tile node n crosses a
// non-periodic side, no node exists at n - e_i; the first step at n writes
// the wall rule of the pull where the second step will read it (the kept
// opposite population plus bbf, or gsign times it plus gconst, the y side
// first at a corner), so the second step reads every node's populations
// with plain LDS loads.  (In the halo layout that place is a slot outside
// the lattice, which no first-step node occupies.)  Halo planes raised the
// 2048^2 step rates by 1.3-5.4% over windows (FP32 D2Q9 thermal the most).
//
// A workgroup has one thread per tile node (64 TY threads), so each phase
// is one pass and the compiler keeps the step constants in scalar
// registers (a loop over rows made it hold them in vector registers, at
// the cost of occupancy).  The kernel is bound by latency more than by
// arithmetic or bandwidth; TY trades halo work against workgroups per CU.
// The fused kernels take TY = 8 (measured on MI355X: FP64 D2Q5 2048^2
// 9.8 TB/s against 9.6 at TY = 4, 4096^2 10.4 against 9.8; with one slot
// per thread, FP32 D2Q5 and both D2Q9 thermal kernels 2-13% faster than
// at TY = 4, which they had taken while two slots per thread limited their
// occupancy), except FP32/FP16 D2Q5, which takes TY = 12: 768-thread
// workgroups, two per CU, 1.20 first-step slots per tile node against
// 1.29, and 1.7% (2048^2), 2.3% (4096^2, strips) and 1.4% (a batch of 256
// cavities) faster; TY = 10 and 16 were 10-18% slower, and TY = 12 cost the
// FP32 flow alone 8% (it keeps 8).
// Each thread steps one first-step slot at a time; the kernels ask the
// compiler for as many waves per SIMD as their LDS allows (fuse2_waves).
// Two slots per thread in flight together held twice the populations in
// registers and cost that occupancy: one slot at a time raised the 2048^2
// and 4096^2 step rates by 1-11% (D2Q9 thermal and the flow alone the most).
// ---------------------------------------------------------------------------
// The value a store to storage type S followed by a load would give.
template <class S>
__device__ __forceinline__ typename Codec<S>::R as_stored(typename Codec<S>::R v, float scale, float inv) {
    if constexpr (std::is_same<S, __half>::value) return __half2float(__float2half_rn(v * scale)) * inv;
    else return v;
}

template <class S, int NG>
struct Fuse2 {
    using R = typename Codec<S>::R;
    static constexpr int NP = 9 + NG;
    static constexpr int TX = 64;
    static constexpr int EW = TX + 2;
#ifdef LBM_FUSE2_ROWS
    static constexpr int TY = LBM_FUSE2_ROWS;   // build-time override of the tile height
#else
    static constexpr int TY = (!std::is_same<S, double>::value && NG == 5) ? 12 : 8;
#endif
    static constexpr int NT = TX * TY;      // threads: one per tile node
    static_assert(NT <= 1024, "a workgroup holds at most 1024 threads");
    static constexpr int EH = TY + 2;
    static constexpr int SLOTS = EW * EH;   // nodes of the first step
    static_assert(SLOTS >= NT, "every thread has a first-step slot");
    // LDS layout.  HALO: plane i holds population i of every slot of the
    // first step (EW x EH, indexed by the slot), so each slot stores all its
    // populations without a test, and tile node n pulls population i from
    // slot n - e_i.  Otherwise plane i holds only the 64 x TY window the
    // tile pulls, indexed by the pulling node; FP64 D2Q9 thermal keeps it,
    // since its halo planes would take more than half the LDS of a CU.
    static constexpr bool HALO = !(std::is_same<S, double>::value && NG == 9);
    static constexpr int PLANE = HALO ? SLOTS : TX * TY;   // LDS values per population
    static_assert(NP * PLANE * (int)sizeof(R) <= 81920, "fused tile needs more than half the LDS of a CU");
};

// LDS index of the value in plane p that tile node (ix, iy) pulls along
// direction i (p = i for the flow, 9 + i for the temperature).
template <class F>
__device__ __forceinline__ int pulled_at(int p, int i, int ix, int iy) {
    if constexpr (F::HALO) return p * F::PLANE + (iy + 1 - ey(i)) * F::EW + (ix + 1 - ex(i));
    else return p * F::PLANE + iy * F::TX + ix;
}

// Slots of the first fused step: the tile and its halo, (sx, sy) in
// [-1, 64] x [-1, TY] relative to the tile origin.  SlotOrder numbers the
// slots that lie in the lattice (or wrap on a periodic axis) so that the
// interior nodes, which pull with the fast path, come first and the nodes
// on the lattice's edge rows and columns, which take the general pull,
// come last: a wave then runs one of the two paths, not both.  The order
// is a permutation of the same slots; results do not depend on it.
struct SlotOrder {
    int cv0, wv, rv0;             // the rectangle of slots in the lattice
    int ci0, ci1, ri0, ri1;       // its interior rectangle
    int n_int, nb, nt, nl;        // interior, bottom, top, left counts
    int wi, wl, wr;               // interior, left and right strip widths
    float inv_wi, inv_wv, inv_wl, inv_wr;
    int count;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// w / d for 0 <= w < 2^12 and 1 <= d < 2^12, with inv = 1 / d: the margin
// of (w + 1/2) / d from an integer (at least 1 / (2d)) dwarfs the rounding
// of the product (below 2^12 / d * 2^-23).
__device__ __forceinline__ int small_div(int w, float inv) { return (int)(((float)w + 0.5f) * inv); }

// The slot grid is EW x EH, the tile grown by MG nodes on every side.
template <int EW, int EH, int MG>
__device__ __forceinline__ SlotOrder slot_order_m(const Geom& G, int x0, int y0) {
    SlotOrder o;
    // slot column l holds x = x0 - MG + l; rows likewise
    const int cv0 = G.px ? 0 : clampi(MG - x0, 0, EW), cv1 = G.px ? EW : clampi(G.nx - x0 + MG, cv0, EW);
    const int rv0 = G.py ? 0 : clampi(MG - y0, 0, EH), rv1 = G.py ? EH : clampi(G.ny - y0 + MG, rv0, EH);
    o.ci0 = clampi(MG + 1 - x0, cv0, cv1);
    o.ci1 = clampi(G.nx - 1 - x0 + MG, o.ci0, cv1);
    o.ri0 = clampi(MG + 1 - y0, rv0, rv1);
    o.ri1 = clampi(G.ny - 1 - y0 + MG, o.ri0, rv1);
    o.cv0 = cv0;
    o.rv0 = rv0;
    o.wv = cv1 - cv0;
    o.wi = o.ci1 - o.ci0;
    o.wl = o.ci0 - cv0;
    o.wr = cv1 - o.ci1;
    const int hi = o.ri1 - o.ri0;
    o.n_int = o.wi * hi;
    o.nb = (o.ri0 - rv0) * o.wv;
    o.nt = (rv1 - o.ri1) * o.wv;
    o.nl = o.wl * hi;
    o.count = o.wv * (rv1 - rv0);
    o.inv_wi = 1.0f / (float)(o.wi > 0 ? o.wi : 1);
    o.inv_wv = 1.0f / (float)(o.wv > 0 ? o.wv : 1);
    o.inv_wl = 1.0f / (float)(o.wl > 0 ? o.wl : 1);
    o.inv_wr = 1.0f / (float)(o.wr > 0 ? o.wr : 1);
    return o;
}

template <class F>
__device__ __forceinline__ SlotOrder slot_order(const Geom& G, int x0, int y0) {
    return slot_order_m<F::EW, F::EH, 1>(G, x0, y0);
}

// Slot coordinates (column l, row m of the slot grid) of work item w < count.
__device__ __forceinline__ void slot_of(const SlotOrder& o, int w, int& l, int& m) {
    int q;
    if (w < o.n_int) {
        q = small_div(w, o.inv_wi);
        l = o.ci0 + w - q * o.wi;
        m = o.ri0 + q;
        return;
    }
    int r = w - o.n_int;
    if (r < o.nb) {
        q = small_div(r, o.inv_wv);
        l = o.cv0 + r - q * o.wv;
        m = o.rv0 + q;
        return;
    }
    r -= o.nb;
    if (r < o.nt) {
        q = small_div(r, o.inv_wv);
        l = o.cv0 + r - q * o.wv;
        m = o.ri1 + q;
        return;
    }
    r -= o.nt;
    if (r < o.nl) {
        q = small_div(r, o.inv_wl);
        l = o.cv0 + r - q * o.wl;
        m = o.ri0 + q;
        return;
    }
    r -= o.nl;
    q = small_div(r, o.inv_wr);
    l = o.ci1 + r - q * o.wr;
    m = o.ri0 + q;
}

// The first fused step on slot (l, m) of the slot grid of a tile at
// (x0, y0): pull (or extrapolate) the pre-collision populations.  Returns
// false for a slot outside a non-periodic side.
template <class S, int NG>
__device__ __forceinline__ bool fuse2_load(const S* __restrict__ src, __amdgpu_buffer_rsrc_t rs, const Geom& G,
                                           const Coeffs& C, int x0, int y0, int l, int m, typename Codec<S>::R f[9],
                                           typename Codec<S>::R g[gdim(NG)]) {
    int x = x0 - 1 + l, y = y0 - 1 + m;
    if (x < 0 || x >= G.nx) {
        if (!G.px) return false;
        x = ((x % G.nx) + G.nx) % G.nx;
    }
    if (y < 0 || y >= G.ny) {
        if (!G.py) return false;
        y = ((y % G.ny) + G.ny) % G.ny;
    }
    if (x >= 1 && x <= G.nx - 2 && y >= 1 && y <= G.ny - 2)
        pull_interior_buf<S, NG>(rs, G, C, (unsigned)(y * G.pitch + x) * (unsigned)sizeof(S), f, g);
    else
        load_node<S, NG>(src, G, C, x, y, f, g);
    return true;
}

// Population I of slot (sx, sy) (tile coordinates) into its window slot
// (window layout only).
template <class S, int NG, int P0, int I>
__device__ __forceinline__ void fuse2_put(typename Codec<S>::R* lds, int sx, int sy, typename Codec<S>::R v) {
    using F = Fuse2<S, NG>;
    const int tx = sx + ex(I), ty = sy + ey(I);
    if (tx >= 0 && tx < F::TX && ty >= 0 && ty < F::TY) lds[(P0 + I) * F::PLANE + ty * F::TX + tx] = v;
}

// The wall rule of link I into tile node (x, y) = (x0 + ix, y0 + iy), if
// the link crosses a non-periodic side; the same arithmetic as the pull.
// It goes where the node pulls that link from: in the halo layout a slot
// outside the lattice, which no first-step node writes.
template <class S, int NG, int I>
__device__ __forceinline__ void fuse2_wall(typename Codec<S>::R* lds, const Geom& G, const Coeffs& C, int x, int y,
                                           int ix, int iy, const typename Codec<S>::R f[9],
                                           const typename Codec<S>::R g[gdim(NG)]) {
    using F = Fuse2<S, NG>;
    using R = typename Codec<S>::R;
    constexpr int dx = ex(I), dy = ey(I);
    const int sx = x - dx, sy = y - dy;
    int side = -1;
    if (dy != 0 && (sy < 0 || sy >= G.ny) && !G.py) side = sy < 0 ? kBottom : kTop;
    if (dx != 0 && (sx < 0 || sx >= G.nx) && !G.px && side < 0) side = sx < 0 ? kLeft : kRight;
    if (side < 0) return;
    lds[pulled_at<F>(I, I, ix, iy)] = f[opp(I)] + (R)C.bbf[side][I];
    if constexpr (I < NG) lds[pulled_at<F>(9 + I, I, ix, iy)] = (R)C.gsign[side] * g[opp(I)] + (R)C.gconst[side][I];
}

template <class S, int NG, int P0, int... I>
__device__ __forceinline__ void fuse2_put_set(typename Codec<S>::R* lds, int sx, int sy,
                                              const typename Codec<S>::R* v, std::integer_sequence<int, I...>) {
    (fuse2_put<S, NG, P0, I>(lds, sx, sy, v[I]), ...);
}

template <class S, int NG, int... I>
__device__ __forceinline__ void fuse2_walls(typename Codec<S>::R* lds, const Geom& G, const Coeffs& C, int x, int y,
                                            int ix, int iy, const typename Codec<S>::R f[9],
                                            const typename Codec<S>::R g[gdim(NG)],
                                            std::integer_sequence<int, I...>) {
    (fuse2_wall<S, NG, I + 1>(lds, G, C, x, y, ix, iy, f, g), ...);
}

// Collide the pulled populations of slot (sl, sm), round them as a store
// to S would, and keep what the second step pulls (no wall rule).
template <class S, int NG, int COLL>
__device__ __forceinline__ void fuse2_keep_open(typename Codec<S>::R* lds, const Coeffs& C, int x0, int y0, int sl,
                                                int sm, typename Codec<S>::R f[9],
                                                typename Codec<S>::R g[gdim(NG)]) {
    using F = Fuse2<S, NG>;
    using R = typename Codec<S>::R;
    const Macro m = macro_at<S, R, NG>(f, g, C, x0 + sl - 1, y0 + sm - 1);
    collide<R, NG, COLL>(f, g, m, C);
    to_stored<S, NG>(f, g, C, y0 + sm - 1);
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = as_stored<S>(f[i], C.fscale, C.finv);
#pragma unroll
    for (int i = 0; i < NG; ++i) g[i] = as_stored<S>(g[i], C.gscale, C.ginv);
    if constexpr (F::HALO) {
        const int at = sm * F::EW + sl;
#pragma unroll
        for (int i = 0; i < 9; ++i) lds[i * F::PLANE + at] = f[i];
#pragma unroll
        for (int i = 0; i < NG; ++i) lds[(9 + i) * F::PLANE + at] = g[i];
    } else {
        fuse2_put_set<S, NG, 0>(lds, sl - 1, sm - 1, f, std::make_integer_sequence<int, 9>{});
        if constexpr (NG > 0) fuse2_put_set<S, NG, 9>(lds, sl - 1, sm - 1, g, std::make_integer_sequence<int, NG>{});
    }
}

// fuse2_keep_open, then the wall rules of the links into a tile node on a
// non-periodic side.
template <class S, int NG, int COLL>
__device__ __forceinline__ void fuse2_keep(typename Codec<S>::R* lds, const Geom& G, const Coeffs& C, int x0, int y0,
                                           int sl, int sm, typename Codec<S>::R f[9],
                                           typename Codec<S>::R g[gdim(NG)]) {
    using F = Fuse2<S, NG>;
    fuse2_keep_open<S, NG, COLL>(lds, C, x0, y0, sl, sm, f, g);
    const int sx = sl - 1, sy = sm - 1;
    const int x = x0 + sx, y = y0 + sy;
    const bool in_tile = sx >= 0 && sx < F::TX && sy >= 0 && sy < F::TY;
    const bool wall = (!G.px && (x == 0 || x == G.nx - 1)) || (!G.py && (y == 0 || y == G.ny - 1));
    if (in_tile && wall) fuse2_walls<S, NG>(lds, G, C, x, y, sx, sy, f, g, std::make_integer_sequence<int, 8>{});
}

// A tile whose every first-step slot (the tile and its halo, x0 - 1 ..
// x0 + TX and y0 - 1 .. y0 + TY) has all its neighbours inside the lattice:
// every slot pulls with the fast path, none is a wall node or wraps, and
// slot w of the row-major slot grid is w itself.  Such "open" tiles run
// the same arithmetic as the general path below without its per-slot
// tests.
template <class F>
__device__ __forceinline__ bool open_tile(const Geom& G, int x0, int y0) {
    return x0 >= 2 && x0 + F::TX <= G.nx - 2 && y0 >= 2 && y0 + F::TY <= G.ny - 2;
}

// The pre-collision populations of slot w of an open tile.
template <class S, int NG>
__device__ __forceinline__ void open_slot_load(__amdgpu_buffer_rsrc_t rs, const Geom& G, const Coeffs& C, int x0,
                                               int y0, int w, typename Codec<S>::R f[9],
                                               typename Codec<S>::R g[gdim(NG)]) {
    using F = Fuse2<S, NG>;
    const int m = w / F::EW, l = w - m * F::EW;
    pull_interior_buf<S, NG>(rs, G, C, (unsigned)((y0 - 1 + m) * G.pitch + (x0 - 1 + l)) * (unsigned)sizeof(S), f, g);
}

// First step of an open tile, the slots of this thread from `first` on
// (earlier ones done by the caller), into LDS.
template <class S, int NG, int COLL>
__device__ __forceinline__ void open_phase1(__amdgpu_buffer_rsrc_t rs, const Geom& G, const Coeffs& C, int x0, int y0,
                                            int first, typename Codec<S>::R* lds) {
    using F = Fuse2<S, NG>;
    using R = typename Codec<S>::R;
#pragma unroll
    for (int w = first; w < F::SLOTS; w += F::NT) {
        R f[9], g[gdim(NG)];
        open_slot_load<S, NG>(rs, G, C, x0, y0, w, f, g);
        const int m = w / F::EW;
        fuse2_keep_open<S, NG, COLL>(lds, C, x0, y0, w - m * F::EW, m, f, g);
    }
}

// First step of a general tile (walls, wraps, lattice edges) into LDS.
template <class S, int NG, int COLL>
__device__ __forceinline__ void general_phase1(__amdgpu_buffer_rsrc_t rs, const S* __restrict__ src, const Geom& G,
                                               const Coeffs& C, int x0, int y0, typename Codec<S>::R* lds) {
    using F = Fuse2<S, NG>;
    using R = typename Codec<S>::R;
    const SlotOrder o = slot_order<F>(G, x0, y0);
    // o.count <= SLOTS: the bound known at compile time fixes the trip count
#pragma unroll
    for (int w = threadIdx.x; w < F::SLOTS; w += F::NT) {
        if (w >= o.count) break;
        R f[9], g[gdim(NG)];
        int l, m;
        slot_of(o, w, l, m);
        if (fuse2_load<S, NG>(src, rs, G, C, x0, y0, l, m, f, g)) fuse2_keep<S, NG, COLL>(lds, G, C, x0, y0, l, m, f, g);
    }
}

// Second step of a tile, pulling from LDS, and the store.  Only wall
// nodes rebuilt by extrapolation read elsewhere: their fluid neighbour's
// pulls, which lie in the tile (the launch rules out one-node edge tiles
// on such sides).  OPEN: the tile is open, no node is a wall node or off
// the lattice.
template <class S, int NG, int MODE, int COLL, bool OPEN>
__device__ __forceinline__ void fused_phase2(__amdgpu_buffer_rsrc_t rd, const Geom& G, const Coeffs& C, int x0, int y0,
                                             const typename Codec<S>::R* lds) {
    using F = Fuse2<S, NG>;
    using R = typename Codec<S>::R;
    const bool inner = (G.px || (x0 > 0 && x0 + F::TX < G.nx)) && (G.py || (y0 > 0 && y0 + F::TY < G.ny));
    const bool nee = !OPEN && C.any_nee && !inner;
#pragma unroll
    for (int n = threadIdx.x; n < F::TX * F::TY; n += F::NT) {
        const int ix = n % F::TX, iy = n / F::TX;
        const int x = x0 + ix, y = y0 + iy;
        if (!OPEN && (x >= G.nx || y >= G.ny)) continue;
        R f[9], g[gdim(NG)];
        if (nee && nee_node_at(G, C, x, y)) {
            const NeeWall w = nee_wall(G, C, x, y);
            const int fx = w.fx - x0, fy = w.fy - y0;
            R ff[9], gf[gdim(NG)];
#pragma unroll
            for (int i = 0; i < 9; ++i) ff[i] = lds[pulled_at<F>(i, i, fx, fy)];
#pragma unroll
            for (int i = 0; i < NG; ++i) gf[i] = lds[pulled_at<F>(9 + i, i, fx, fy)];
            nee_rebuild<R, NG>(w, C, ff, gf, f, g);
        } else {
#pragma unroll
            for (int i = 0; i < 9; ++i) f[i] = lds[pulled_at<F>(i, i, ix, iy)];
#pragma unroll
            for (int i = 0; i < NG; ++i) g[i] = lds[pulled_at<F>(9 + i, i, ix, iy)];
        }
        const Macro m = macro_at<S, R, NG>(f, g, C, x, y);
        collide<R, NG, COLL>(f, g, m, C);
        to_stored<S, NG>(f, g, C, y);
        const unsigned boff = (unsigned)(y * G.pitch + x) * (unsigned)sizeof(S);
        if (MODE == kBufferKeep) store_node_buf<S, NG, kCachePolicyDefault>(rd, G, C, boff, f, g);
        else store_node_buf<S, NG, kCachePolicyNT>(rd, G, C, boff, f, g);
    }
}

// One fused pair of steps on the tile at (x0, y0) of one lattice (the
// batch kernel's body).
template <class S, int NG, int MODE, int COLL>
__device__ __forceinline__ void fused_tile(const Geom& G, const Coeffs& C, const S* __restrict__ src,
                                           S* __restrict__ dst, unsigned buf_bytes, int x0, int y0,
                                           typename Codec<S>::R* lds) {
    using F = Fuse2<S, NG>;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(src, buf_bytes);
    const __amdgpu_buffer_rsrc_t rd = make_rsrc(dst, buf_bytes);
    if (open_tile<F>(G, x0, y0)) {
        open_phase1<S, NG, COLL>(rs, G, C, x0, y0, threadIdx.x, lds);
        __syncthreads();
        fused_phase2<S, NG, MODE, COLL, true>(rd, G, C, x0, y0, lds);
    } else {
        general_phase1<S, NG, COLL>(rs, src, G, C, x0, y0, lds);
        __syncthreads();
        fused_phase2<S, NG, MODE, COLL, false>(rd, G, C, x0, y0, lds);
    }
}

// Waves per SIMD the fused kernels ask the compiler for: what their LDS
// allows per CU (FP64 D2Q5 is bound by its LDS at four and asks nothing).
// FP64: 6 without temperature, 4 for D2Q9 thermal (a 28-byte spill);
// FP32/FP16: 8, 6 and 4.  FP32/FP16 D2Q5 stops at 6 below the 8 its LDS
// would allow: at 8 it spills 35 VGPRs for a 1% faster step on MI355X.
template <class S>
constexpr int fuse2_waves(int NG) {
    return std::is_same<S, double>::value ? (NG == 0 ? 6 : (NG == 9 ? 4 : 1)) : (NG == 0 ? 8 : (NG == 5 ? 6 : 4));
}

template <class S, int NG, int MODE, int COLL>
__global__ __launch_bounds__((Fuse2<S, NG>::NT)) __attribute__((amdgpu_waves_per_eu(fuse2_waves<S>(NG), 8))) void k_sweep2(
    Geom G, const Coeffs* __restrict__ Cp, const S* __restrict__ src, S* __restrict__ dst, int tiles_x,
    unsigned buf_bytes, int order) {
    using F = Fuse2<S, NG>;
    __shared__ typename Codec<S>::R lds[F::NP * F::PLANE];
    const int tile = xcd_remap(blockIdx.x, gridDim.x, order, tiles_x);
    fused_tile<S, NG, MODE, COLL>(G, *Cp, src, dst, buf_bytes, (tile % tiles_x) * F::TX, (tile / tiles_x) * F::TY,
                                  lds);
}

// Fused pairs of steps for every lattice of a batch: each workgroup takes
// one entry of the fused tile table (a member and its 64 x TY tile).
template <class S, int NG, int MODE>
__global__ __launch_bounds__((Fuse2<S, NG>::NT)) __attribute__((amdgpu_waves_per_eu(fuse2_waves<S>(NG), 8)))
void k_sweep2_batch(
    const BatchMember* __restrict__ members, const BatchTile* __restrict__ tiles, int parity, int order) {
    using F = Fuse2<S, NG>;
    __shared__ typename Codec<S>::R lds[F::NP * F::PLANE];
    const BatchTile t = tiles[xcd_remap(blockIdx.x, gridDim.x, order, 0)];
    const BatchMember& M = members[t.member];
    const int sel = (M.cur0 + parity) & 1;
    fused_tile<S, NG, MODE, kCollMRT>(M.G, M.C, static_cast<const S*>(M.buf[sel]), static_cast<S*>(M.buf[sel ^ 1]),
                                      M.buf_bytes, t.x0, t.y0, lds);
}

// ---------------------------------------------------------------------------
// K >= 3 time steps per launch.  A workgroup owns a TX x TY tile.  Step 1
// runs on the tile grown by K - 1 nodes on every side, reading the state
// from HBM as the single-step kernel does; step s runs on the tile grown by
// K - s nodes, pulling the post-collision populations of step s - 1 from
// LDS; step K runs on the tile and stores to HBM.  The state crosses HBM
// once per K steps; the margins cost sum_s (TX + 2(K - s))(TY + 2(K - s)) /
// (TX TY K) - 1 extra collisions per node and step.  The result is bitwise
// the result of K single steps.
//
// LDS holds one plane per population over the region of step 2 (the tile
// grown by K - 2 nodes), indexed by the pulling node: a node of step s >= 2
// reads every population at its own index; a node of step s - 1 writes
// population i at the index of the node that pulls it, its own position +
// e_i, when that node takes part in step s.  With one buffer (FP64) steps
// 2 .. K - 1 update the planes in place: every node reads and collides, a
// barrier, then every node writes (each index has one writer and one reader
// per step); with two (FP32) they read one buffer and write the other.  Where
// the link into a node of step s crosses a non-periodic side, no node
// exists at its source; the node itself writes the wall rule of the pull at
// its own index in that plane in step s - 1, the one index of the plane no
// other node writes.  Wall nodes rebuilt by extrapolation read their fluid
// neighbour's pulls, which lie in the same step's region (the launch rules
// out one-node edge tiles on such sides).  Generic over the storage; built
// for FP64 and FP32 (fusek_built).
// ---------------------------------------------------------------------------
template <class S, int NG, int K, int TY_, int TX_>
struct FuseK {
    using R = typename Codec<S>::R;
    using Store = S;
    static_assert(K >= 3, "two steps per launch are the fused pair");
    static constexpr int NP = 9 + NG;
    static constexpr int TX = TX_;
    static constexpr int TY = TY_;
    static constexpr int NT = TX * TY;          // threads: one per tile node
    static_assert(NT <= 1024, "a workgroup holds at most 1024 threads");
    static constexpr int WM = K - 2;            // margin of the LDS window (step 2's region)
    static constexpr int WX = TX + 2 * WM, WY = TY + 2 * WM;
    static constexpr int PLANE = WX * WY;
    static constexpr int M1 = K - 1;            // margin of the first step
    static constexpr int E1X = TX + 2 * M1, E1Y = TY + 2 * M1;
    static constexpr int SLOTS1 = E1X * E1Y;
    // Two LDS buffers (the middle steps read one and write the other, no
    // results held across a barrier) where both fit in half a CU's LDS
    // (FP32: 2048^2 step 43.0 against 44.2 us with one buffer in place);
    // otherwise one, updated in place (FP64).
    static constexpr bool DB = 2 * NP * PLANE * (int)sizeof(R) <= 81920;
    static constexpr int LDS_VALUES = (DB ? 2 : 1) * NP * PLANE;
    static_assert(LDS_VALUES * (int)sizeof(R) <= 81920, "fused tile needs more than half the LDS of a CU");
    // workgroups per CU the LDS (160 KiB) and the CU's 32 wave slots allow
    static constexpr int WG_PER_CU = (163840 / (LDS_VALUES * (int)sizeof(R)) < 2048 / NT)
                                         ? 163840 / (LDS_VALUES * (int)sizeof(R)) : 2048 / NT;
    // LDS index of plane p at the node (sx, sy) relative to the tile origin
    static __device__ __forceinline__ int at(int p, int sx, int sy) { return p * PLANE + (sy + WM) * WX + (sx + WM); }
};

// Whether tile-relative (sx, sy) lies in the tile grown by MG nodes.
template <class F, int MG>
__device__ __forceinline__ bool in_region(int sx, int sy) {
    return sx >= -MG && sx < F::TX + MG && sy >= -MG && sy < F::TY + MG;
}

// Population I of the node at (sx, sy) to the node (sx, sy) + e_I that
// pulls it, if that node takes part in the next step (region of margin MN).
template <class F, int MN, int P0, int I>
__device__ __forceinline__ void fk_put(typename F::R* lds, int sx, int sy, typename F::R v) {
    const int tx = sx + ex(I), ty = sy + ey(I);
    if (in_region<F, MN>(tx, ty)) lds[F::at(P0 + I, tx, ty)] = v;
}

template <class F, int MN, int P0, int... I>
__device__ __forceinline__ void fk_put_set(typename F::R* lds, int sx, int sy, const typename F::R* v,
                                           std::integer_sequence<int, I...>) {
    (fk_put<F, MN, P0, I>(lds, sx, sy, v[I]), ...);
}

// The wall rule of link I into lattice node (x, y), at tile-relative
// (sx, sy), if the link crosses a non-periodic side (the arithmetic of the
// pull); it goes to the node's own index in plane I.
template <class F, int NG, int I>
__device__ __forceinline__ void fk_wall(typename F::R* lds, const Geom& G, const Coeffs& C, int x, int y, int sx,
                                        int sy, const typename F::R f[9], const typename F::R g[gdim(NG)]) {
    using R = typename F::R;
    constexpr int dx = ex(I), dy = ey(I);
    const int px = x - dx, py = y - dy;
    int side = -1;
    if (dy != 0 && (py < 0 || py >= G.ny) && !G.py) side = py < 0 ? kBottom : kTop;
    if (dx != 0 && (px < 0 || px >= G.nx) && !G.px && side < 0) side = px < 0 ? kLeft : kRight;
    if (side < 0) return;
    lds[F::at(I, sx, sy)] = f[opp(I)] + (R)C.bbf[side][I];
    if constexpr (I < NG) lds[F::at(9 + I, sx, sy)] = (R)C.gsign[side] * g[opp(I)] + (R)C.gconst[side][I];
}

template <class F, int NG, int... I>
__device__ __forceinline__ void fk_walls(typename F::R* lds, const Geom& G, const Coeffs& C, int x, int y, int sx,
                                         int sy, const typename F::R f[9], const typename F::R g[gdim(NG)],
                                         std::integer_sequence<int, I...>) {
    (fk_wall<F, NG, I + 1>(lds, G, C, x, y, sx, sy, f, g), ...);
}

// The post-collision populations of lattice node (x, y) at tile-relative
// (sx, sy) into LDS for the next step, whose region has margin MN: in the
// form and rounding a store and a load of the storage type would give
// them (FP16: relative to the reference of the pulling node), each to the
// node that pulls it and, with WALLS, the wall rules of the node's own
// links if it takes part in the next step.
template <class F, int NG, int MN, bool WALLS>
__device__ __forceinline__ void fk_keep(typename F::R* lds, const Geom& G, const Coeffs& C, int x, int y, int sx,
                                        int sy, typename F::R f[9], typename F::R g[gdim(NG)]) {
    using S = typename F::Store;
    to_stored<S, NG>(f, g, C, y);
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = as_stored<S>(f[i], C.fscale, C.finv);
#pragma unroll
    for (int i = 0; i < NG; ++i) g[i] = as_stored<S>(g[i], C.gscale, C.ginv);
    fk_put_set<F, MN, 0>(lds, sx, sy, f, std::make_integer_sequence<int, 9>{});
    if constexpr (NG > 0) fk_put_set<F, MN, 9>(lds, sx, sy, g, std::make_integer_sequence<int, NG>{});
    if constexpr (WALLS) {
        const bool wall = (!G.px && (x == 0 || x == G.nx - 1)) || (!G.py && (y == 0 || y == G.ny - 1));
        if (wall && in_region<F, MN>(sx, sy))
            fk_walls<F, NG>(lds, G, C, x, y, sx, sy, f, g, std::make_integer_sequence<int, 8>{});
    }
}

// Pre-collision populations of a node of step s >= 2 at tile-relative
// (sx, sy), lattice (x, y), from LDS: its own index, or, for a wall node
// rebuilt by extrapolation (NEE), its fluid neighbour's.
template <class F, int NG, bool NEE>
__device__ __forceinline__ void fk_read(const typename F::R* lds, const Geom& G, const Coeffs& C, int x, int y, int sx,
                                        int sy, typename F::R f[9], typename F::R g[gdim(NG)]) {
    using R = typename F::R;
    if (NEE && nee_node_at(G, C, x, y)) {
        const NeeWall w = nee_wall(G, C, x, y);
        const int fx = sx + (w.fx - x), fy = sy + (w.fy - y);
        R ff[9], gf[gdim(NG)];
#pragma unroll
        for (int i = 0; i < 9; ++i) ff[i] = lds[F::at(i, fx, fy)];
#pragma unroll
        for (int i = 0; i < NG; ++i) gf[i] = lds[F::at(9 + i, fx, fy)];
        nee_rebuild<R, NG>(w, C, ff, gf, f, g);
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = lds[F::at(i, sx, sy)];
#pragma unroll
        for (int i = 0; i < NG; ++i) g[i] = lds[F::at(9 + i, sx, sy)];
    }
}

// Lattice coordinate of tile-relative position v along an axis of n nodes
// starting at v0; false outside a non-periodic axis.
__device__ __forceinline__ bool fk_axis(int v0, int v, int n, int periodic, int& out) {
    int a = v0 + v;
    if (a < 0 || a >= n) {
        if (!periodic) return false;
        a = ((a % n) + n) % n;
    }
    out = a;
    return true;
}

// Step 1 of a general tile (walls, wraps, lattice edges) from HBM into LDS,
// slots in interior-first order.
template <class S, int NG, class F, int COLL>
__device__ __forceinline__ void fk_first_general(__amdgpu_buffer_rsrc_t rs, const S* __restrict__ src, const Geom& G,
                                                 const Coeffs& C, int x0, int y0, typename F::R* lds) {
    using R = typename F::R;
    const SlotOrder o = slot_order_m<F::E1X, F::E1Y, F::M1>(G, x0, y0);
    if constexpr (!std::is_same<S, double>::value) {
        // FP32: one slot at a time (issuing every slot's fast pulls first
        // made the 2048^2 step 3% slower on MI355X)
#pragma unroll
        for (int w = threadIdx.x; w < F::SLOTS1; w += F::NT) {
            if (w >= o.count) break;
            int l, m;
            slot_of(o, w, l, m);
            const int sx = l - F::M1, sy = m - F::M1;
            int x, y;
            if (!fk_axis(x0, sx, G.nx, G.px, x) || !fk_axis(y0, sy, G.ny, G.py, y)) continue;
            R f[9], g[gdim(NG)];
            if (x >= 1 && x <= G.nx - 2 && y >= 1 && y <= G.ny - 2)
                pull_interior_buf<S, NG>(rs, G, C, (unsigned)(y * G.pitch + x) * (unsigned)sizeof(S), f, g);
            else
                load_node<S, NG>(src, G, C, x, y, f, g);
            const Macro mc = macro_at<S, R, NG>(f, g, C, x, y);
            collide<R, NG, COLL>(f, g, mc, C);
            fk_keep<F, NG, F::WM, true>(lds, G, C, x, y, sx, sy, f, g);
        }
        return;
    }
    // FP64: the fast pulls of every slot are issued before the first
    // collision (interior slots come first in the order; 4096^2 step 5%
    // faster on MI355X); edge slots pull per link in the second pass
    constexpr int P = (F::SLOTS1 + F::NT - 1) / F::NT;
    R f[P][9], g[P][gdim(NG)];
    int xs[P], ys[P], sxs[P], sys[P];
    bool ok[P], fast[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const int w = (int)threadIdx.x + k * F::NT;
        ok[k] = w < o.count;
        fast[k] = false;
        xs[k] = ys[k] = sxs[k] = sys[k] = 0;
        if (ok[k]) {
            int l, m;
            slot_of(o, w, l, m);
            sxs[k] = l - F::M1;
            sys[k] = m - F::M1;
            ok[k] = fk_axis(x0, sxs[k], G.nx, G.px, xs[k]) && fk_axis(y0, sys[k], G.ny, G.py, ys[k]);
        }
        if (ok[k]) {
            const int x = xs[k], y = ys[k];
            fast[k] = x >= 1 && x <= G.nx - 2 && y >= 1 && y <= G.ny - 2;
            if (fast[k])
                pull_interior_buf<S, NG>(rs, G, C, (unsigned)(y * G.pitch + x) * (unsigned)sizeof(S), f[k], g[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
        if (!ok[k]) continue;
        if (!fast[k]) load_node<S, NG>(src, G, C, xs[k], ys[k], f[k], g[k]);
        const Macro mc = macro_at<S, R, NG>(f[k], g[k], C, xs[k], ys[k]);
        collide<R, NG, COLL>(f[k], g[k], mc, C);
        fk_keep<F, NG, F::WM, true>(lds, G, C, xs[k], ys[k], sxs[k], sys[k], f[k], g[k]);
    }
}

// Step 1 of an open tile (every slot pulls with the fast path; no wall node,
// no wrap) from HBM into LDS.
template <class S, int NG, class F, int COLL>
__device__ __forceinline__ void fk_first_open(__amdgpu_buffer_rsrc_t rs, const Geom& G, const Coeffs& C, int x0,
                                              int y0, typename F::R* lds) {
    using R = typename F::R;
    // every slot's loads are issued before the first collision: the thread
    // keeps P slots' worth of bytes in flight instead of one
    constexpr int P = (F::SLOTS1 + F::NT - 1) / F::NT;
    R f[P][9], g[P][gdim(NG)];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const int w = (int)threadIdx.x + k * F::NT;
        if (w < F::SLOTS1) {
            const int m = w / F::E1X, l = w - m * F::E1X;
            const int x = x0 + l - F::M1, y = y0 + m - F::M1;
            pull_interior_buf<S, NG>(rs, G, C, (unsigned)(y * G.pitch + x) * (unsigned)sizeof(S), f[k], g[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const int w = (int)threadIdx.x + k * F::NT;
        if (w < F::SLOTS1) {
            const int m = w / F::E1X, l = w - m * F::E1X;
            const int sx = l - F::M1, sy = m - F::M1;
            const int x = x0 + sx, y = y0 + sy;
            const Macro mc = macro_at<S, R, NG>(f[k], g[k], C, x, y);
            collide<R, NG, COLL>(f[k], g[k], mc, C);
            fk_keep<F, NG, F::WM, false>(lds, G, C, x, y, sx, sy, f[k], g[k]);
        }
    }
}

// A middle step (2 .. K - 1) on the tile grown by MG nodes.  With one LDS
// buffer (in == out) it runs in place: every node reads and collides, then
// (after a barrier) writes for the step on the tile grown by MG - 1, each
// thread holding the results of its nodes across the barrier.  With two,
// each node reads `in` and writes `out` at once.  Ends with a barrier.
template <class S, int NG, class F, int COLL, int MG, bool OPEN>
__device__ __forceinline__ void fk_middle(const Geom& G, const Coeffs& C, int x0, int y0,
                                          const typename F::R* in, typename F::R* out) {
    using R = typename F::R;
    constexpr int RX = F::TX + 2 * MG, RY = F::TY + 2 * MG, N = RX * RY;
    const bool nee = !OPEN && C.any_nee;
    if constexpr (F::DB) {
#pragma unroll
        for (int w = threadIdx.x; w < N; w += F::NT) {
            const int sy = w / RX - MG, sx = w - (sy + MG) * RX - MG;
            int x = x0 + sx, y = y0 + sy;
            if (!OPEN && !(fk_axis(x0, sx, G.nx, G.px, x) && fk_axis(y0, sy, G.ny, G.py, y))) continue;
            R f[9], g[gdim(NG)];
            if (nee) fk_read<F, NG, true>(in, G, C, x, y, sx, sy, f, g);
            else fk_read<F, NG, false>(in, G, C, x, y, sx, sy, f, g);
            const Macro mc = macro_at<S, R, NG>(f, g, C, x, y);
            collide<R, NG, COLL>(f, g, mc, C);
            fk_keep<F, NG, MG - 1, !OPEN>(out, G, C, x, y, sx, sy, f, g);
        }
        __syncthreads();
        return;
    }
    typename F::R* lds = out;
    constexpr int P = (N + F::NT - 1) / F::NT;
    R f[P][9], g[P][gdim(NG)];
    int xs[P], ys[P];
    bool ok[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const int w = (int)threadIdx.x + k * F::NT;
        const int sy = w / RX - MG, sx = w - (sy + MG) * RX - MG;
        int x = x0 + sx, y = y0 + sy;
        ok[k] = w < N;
        if (!OPEN && ok[k]) ok[k] = fk_axis(x0, sx, G.nx, G.px, x) && fk_axis(y0, sy, G.ny, G.py, y);
        xs[k] = x;
        ys[k] = y;
        if (ok[k]) {
            if (nee) fk_read<F, NG, true>(lds, G, C, x, y, sx, sy, f[k], g[k]);
            else fk_read<F, NG, false>(lds, G, C, x, y, sx, sy, f[k], g[k]);
            const Macro mc = macro_at<S, R, NG>(f[k], g[k], C, x, y);
            collide<R, NG, COLL>(f[k], g[k], mc, C);
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const int w = (int)threadIdx.x + k * F::NT;
        const int sy = w / RX - MG, sx = w - (sy + MG) * RX - MG;
        if (ok[k]) fk_keep<F, NG, MG - 1, !OPEN>(lds, G, C, xs[k], ys[k], sx, sy, f[k], g[k]);
    }
    __syncthreads();
}

// The middle steps, margins K - 2 down to 1 (J = 0 .. K - 3); with two
// buffers step J reads buffer J % 2 and writes the other.
template <class S, int NG, class F, int COLL, bool OPEN, int... J>
__device__ __forceinline__ void fk_middles(const Geom& G, const Coeffs& C, int x0, int y0, typename F::R* lds,
                                           std::integer_sequence<int, J...>) {
    constexpr int B = F::NP * F::PLANE;
    (fk_middle<S, NG, F, COLL, F::WM - J, OPEN>(G, C, x0, y0, lds + (F::DB ? (J % 2) * B : 0),
                                                 lds + (F::DB ? ((J + 1) % 2) * B : 0)),
     ...);
}

// The buffer the last step reads.
template <class F>
__device__ __forceinline__ const typename F::R* fk_last_buffer(const typename F::R* lds) {
    constexpr int K = F::M1 + 1;
    return lds + (F::DB ? ((K - 2) % 2) * F::NP * F::PLANE : 0);
}

// The last step on the tile, pulling from LDS, and the store.
template <class S, int NG, class F, int MODE, int COLL, bool OPEN>
__device__ __forceinline__ void fk_last(__amdgpu_buffer_rsrc_t rd, const Geom& G, const Coeffs& C, int x0, int y0,
                                        const typename F::R* lds) {
    using R = typename F::R;
    const int ix = (int)threadIdx.x % F::TX, iy = (int)threadIdx.x / F::TX;
    const int x = x0 + ix, y = y0 + iy;
    if (!OPEN && (x >= G.nx || y >= G.ny)) return;
    R f[9], g[gdim(NG)];
    if (!OPEN && C.any_nee) fk_read<F, NG, true>(lds, G, C, x, y, ix, iy, f, g);
    else fk_read<F, NG, false>(lds, G, C, x, y, ix, iy, f, g);
    const Macro m = macro_at<S, R, NG>(f, g, C, x, y);
    collide<R, NG, COLL>(f, g, m, C);
    to_stored<S, NG>(f, g, C, y);
    const unsigned boff = (unsigned)(y * G.pitch + x) * (unsigned)sizeof(S);
    if (MODE == kBufferKeep) store_node_buf<S, NG, kCachePolicyDefault>(rd, G, C, boff, f, g);
    else store_node_buf<S, NG, kCachePolicyNT>(rd, G, C, boff, f, g);
}

template <class F>
__device__ __forceinline__ bool fk_open_tile(const Geom& G, int x0, int y0) {
    constexpr int K = F::M1 + 1;
    return x0 >= K && x0 + F::TX <= G.nx - K && y0 >= K && y0 + F::TY <= G.ny - K;
}

// Time steps per launch of the multi-step kernel and its tile.  Four steps
// on 32 x 16 tiles: the FP64 D2Q5 window (14 planes of 36 x 20) takes
// 80.6 KB, so two workgroups share a CU, and a launch collides 5.23 times
// per tile node (1.31 per step).  Measured on MI355X (2048^2 heated cavity,
// FP64, per step): 55.7 us against 63.8 for three steps on 64 x 8 tiles
// (4096^2 200.8 against 238.6; the flow alone 38.0 against 44.4; FP32 42.0
// against 43.6).  The tile shape alone gains nothing: three steps on
// 32 x 16 or 32 x 8 tiles (four workgroups per CU) took 64.8 us each,
// on 32 x 12 (three per CU, spilling) 82.5; four steps on 64 x 8 tiles
// would need 91 KB for FP64, one workgroup per CU, and took 45.0 against
// 42.4 us per FP32 step, its window updated in place.  The D2Q9 thermal
// model (18 planes) takes three steps on 32 x 8 tiles: a 49 KB FP64 window,
// three workgroups per CU; 2048^2 FP64 85.7 against 108.8 us per step for
// fused pairs (4096^2 323.0 against 409.9, 1024^2 26.2 against 31.3).  The
// kernel takes any K >= 3 and any tile whose window fits half the LDS.
template <class S, int NG>
constexpr int fusek_steps() {
    return NG == 9 ? 3 : 4;
}

template <class S, int NG, int K>
constexpr int fusek_rows() {
    return NG == 9 ? 8 : 16;
}

template <class S, int NG, int K>
constexpr int fusek_cols() {
    return 32;
}

template <class S, int NG, int K>
using FuseKT = FuseK<S, NG, K, fusek_rows<S, NG, K>(), fusek_cols<S, NG, K>()>;

// Waves per SIMD for as many workgroups per CU as the LDS allows, asked of
// the compiler so that its register budget lets them in.
template <class S, int NG, int K>
constexpr int fusek_waves() {
    constexpr int w = (FuseKT<S, NG, K>::WG_PER_CU * FuseKT<S, NG, K>::NT / 64 + 3) / 4;
    return w < 8 ? w : 8;
}

// K fused steps on the tile at (x0, y0) of one lattice (the body of the
// single-lattice and batch kernels).
template <class S, int NG, int K, int MODE, int COLL>
__device__ __forceinline__ void fusek_tile(const Geom& G, const Coeffs& C, const S* __restrict__ src,
                                           S* __restrict__ dst, unsigned buf_bytes, int x0, int y0,
                                           typename Codec<S>::R* lds) {
    using F = FuseKT<S, NG, K>;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(src, buf_bytes);
    const __amdgpu_buffer_rsrc_t rd = make_rsrc(dst, buf_bytes);
    if (fk_open_tile<F>(G, x0, y0)) {
        fk_first_open<S, NG, F, COLL>(rs, G, C, x0, y0, lds);
        __syncthreads();
        fk_middles<S, NG, F, COLL, true>(G, C, x0, y0, lds, std::make_integer_sequence<int, K - 2>{});
        fk_last<S, NG, F, MODE, COLL, true>(rd, G, C, x0, y0, fk_last_buffer<F>(lds));
    } else {
        fk_first_general<S, NG, F, COLL>(rs, src, G, C, x0, y0, lds);
        __syncthreads();
        fk_middles<S, NG, F, COLL, false>(G, C, x0, y0, lds, std::make_integer_sequence<int, K - 2>{});
        fk_last<S, NG, F, MODE, COLL, false>(rd, G, C, x0, y0, fk_last_buffer<F>(lds));
    }
}

template <class S, int NG, int K, int MODE, int COLL>
__global__ __launch_bounds__((FuseKT<S, NG, K>::NT))
__attribute__((amdgpu_waves_per_eu(fusek_waves<S, NG, K>(), 8))) void k_sweepk(
    Geom G, const Coeffs* __restrict__ Cp, const S* __restrict__ src, S* __restrict__ dst, int tiles_x,
    unsigned buf_bytes, int order) {
    using F = FuseKT<S, NG, K>;
    __shared__ typename F::R lds[F::LDS_VALUES];
    const int tile = xcd_remap(blockIdx.x, gridDim.x, order, tiles_x);
    fusek_tile<S, NG, K, MODE, COLL>(G, *Cp, src, dst, buf_bytes, (tile % tiles_x) * F::TX, (tile / tiles_x) * F::TY,
                                     lds);
}

// K fused steps for every lattice of a batch: each workgroup takes one
// entry of the K-step tile table (a member and its TX x TY tile).
template <class S, int NG, int K, int MODE>
__global__ __launch_bounds__((FuseKT<S, NG, K>::NT))
__attribute__((amdgpu_waves_per_eu(fusek_waves<S, NG, K>(), 8))) void k_sweepk_batch(
    const BatchMember* __restrict__ members, const BatchTile* __restrict__ tiles, int parity, int order) {
    using F = FuseKT<S, NG, K>;
    __shared__ typename F::R lds[F::LDS_VALUES];
    const BatchTile t = tiles[xcd_remap(blockIdx.x, gridDim.x, order, 0)];
    const BatchMember& M = members[t.member];
    const int sel = (M.cur0 + parity) & 1;
    fusek_tile<S, NG, K, MODE, kCollMRT>(M.G, M.C, static_cast<const S*>(M.buf[sel]), static_cast<S*>(M.buf[sel ^ 1]),
                                         M.buf_bytes, t.x0, t.y0, lds);
}

// One time step of every lattice of a batch.  Each workgroup of 256
// threads takes one entry of the tile table: a member lattice and a tile
// of bx x (256 / bx) nodes at (x0, y0).  Member m reads buffer
// (cur0 + parity) & 1 and writes the other one.
template <class S, int NG, int MODE>
__global__ __launch_bounds__(256) void k_sweep_batch(const BatchMember* __restrict__ members,
                                                     const BatchTile* __restrict__ tiles, int parity, int order) {
    const BatchTile t = tiles[xcd_remap(blockIdx.x, gridDim.x, order, 0)];
    const BatchMember& M = members[t.member];
    const int sel = (M.cur0 + parity) & 1;
    const S* src = static_cast<const S*>(M.buf[sel]);
    S* dst = static_cast<S*>(M.buf[sel ^ 1]);
    const int x = t.x0 + (int)(threadIdx.x % (unsigned)t.bx);
    const int y = t.y0 + (int)(threadIdx.x / (unsigned)t.bx);
    sweep_nodes<S, NG, 1, MODE, kCollMRT>(M.G, M.C, src, dst, x, y, M.buf_bytes);
}

template <class S, int NG>
__global__ __launch_bounds__(256) void k_moments(Geom G, Coeffs C, const S* __restrict__ src, double* rho,
                                                 double* ux, double* uy, double* T) {
    using R = typename Codec<S>::R;
    const long long n = (long long)G.nx * G.ny;
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int x = (int)(k % G.nx), y = (int)(k / G.nx);
    R f[9], g[gdim(NG)];
    load_node<S, NG>(src, G, C, x, y, f, g);
    const Macro m = macro_at<S, R, NG>(f, g, C, x, y);
    if (rho) rho[k] = Codec<S>::kDev ? 1.0 + rref_at<S>(C, y) + m.rho : m.rho;
    if (ux) ux[k] = m.ux;
    if (uy) uy[k] = m.uy;
    if (T) T[k] = m.T;
}

// Rest populations that deviation storage subtracts: w_i rho0 for fbar,
// g_i^eq(T0, 0) for g (Eq. 30 for D2Q5, Eq. 31 for D2Q9).
__device__ __forceinline__ double rest_f(int i) { return w9(i); }
template <int NG>
__device__ __forceinline__ double rest_g(int i, double T, double varpi) {
    if constexpr (NG == 5) return i == 0 ? (1.0 - varpi) * T : 0.25 * varpi * T;
    else return w9(i) * T;
}

template <class S, int NG>
__global__ __launch_bounds__(256) void k_gather(Geom G, Coeffs C, const S* __restrict__ src, double* pf,
                                                double* pg, double T0) {
    using R = typename Codec<S>::R;
    const long long n = (long long)G.nx * G.ny;
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int x = (int)(k % G.nx), y = (int)(k / G.nx);
    R f[9], g[gdim(NG)];
    load_node<S, NG>(src, G, C, x, y, f, g);
    constexpr bool dev = Codec<S>::kDev;
    if (pf)
        for (int i = 0; i < 9; ++i)
            pf[i * n + k] = dev ? rest_f(i) * (1.0 + rref_at<S>(C, y)) + (double)f[i] : (double)f[i];
    if (pg)
        for (int i = 0; i < NG; ++i)
            pg[i * n + k] = dev ? rest_g<NG>(i, T0 + tref_at<S>(C, x, y), C.varpi) + (double)g[i] : (double)g[i];
}

// Destination of the stored entry (i, x, y) under the pull: the node
// (x + e_i, y + e_i) if the link stays inside (after periodic wrap), else
// the wall it crosses (y walls first, as in source()).
template <int I>
__device__ __forceinline__ int target(const Geom& G, int x, int y, int& tx, int& ty) {
    int sx = x + ex(I), sy = y + ey(I), side = -1;
    if (ey(I) != 0 && (sy < 0 || sy >= G.ny)) {
        if (G.py) sy = sy < 0 ? sy + G.ny : sy - G.ny;
        else side = sy < 0 ? kBottom : kTop;
    }
    if (ex(I) != 0 && (sx < 0 || sx >= G.nx)) {
        if (G.px) sx = sx < 0 ? sx + G.nx : sx - G.nx;
        else if (side < 0) side = sx < 0 ? kLeft : kRight;
    }
    tx = sx;
    ty = sy;
    return side;
}

// Pre-collision value of population i at node k, in the stored
// representation (full for FP64, deviation otherwise).
// MODE 0: from FP64 arrays pf/pg ([i][node]); MODE 1: rest equilibrium
// with the temperature field Tf (or T0 if Tf is null), Eqs. 22, 30, 31.
// Deviations are relative to the node's reference state: temperature
// T0 + tau, density rho0 + rho_ref (both zero but for FP16; tb, tgx, tgy,
// r0, rA, rB of Coeffs, nx the lattice width).
template <bool DEV, int NG, int MODE>
struct PreValue {
    const double *pf, *pg, *Tf;
    long long n;
    double T0, varpi;
    double tb, tgx, tgy;
    double r0, rA, rB;
    int nx;
    __device__ double tau(long long k) const {
        return tb + tgx * (double)(k % nx) + tgy * (double)(k / nx);
    }
    __device__ double rho_ref(long long k) const {
        const double y = (double)(k / nx);
        return r0 + rA * y + rB * y * y;
    }
    __device__ double f(int i, long long k) const {
        if (MODE == 0) return DEV ? pf[i * n + k] - rest_f(i) * (1.0 + rho_ref(k)) : pf[i * n + k];
        return DEV ? 0.0 - rest_f(i) * rho_ref(k) : rest_f(i);
    }
    __device__ double g(int i, long long k) const {
        if (MODE == 0) return DEV ? pg[i * n + k] - rest_g<NG>(i, T0 + tau(k), varpi) : pg[i * n + k];
        const double T = Tf ? Tf[k] : T0;
        return rest_g<NG>(i, DEV ? T - T0 - tau(k) : T, varpi);
    }
};

template <class S, int NG, int MODE, int I>
__device__ __forceinline__ void unstream_f(S* __restrict__ dst, const Geom& G, const Coeffs& C,
                                           const PreValue<Codec<S>::kDev, NG, MODE>& pv, int x, int y, long long k,
                                           long long o) {
    using R = typename Codec<S>::R;
    int tx, ty;
    const int side = target<I>(G, x, y, tx, ty);
    const double v = side < 0 ? pv.f(I, (long long)ty * G.nx + tx) : pv.f(opp(I), k) - C.bbf[side][opp(I)];
    Codec<S>::store(dst + (long long)I * G.plane + o, (R)v, C.fscale);
}

template <class S, int NG, int MODE, int I>
__device__ __forceinline__ void unstream_g(S* __restrict__ dst, const Geom& G, const Coeffs& C,
                                           const PreValue<Codec<S>::kDev, NG, MODE>& pv, int x, int y, long long k,
                                           long long o) {
    using R = typename Codec<S>::R;
    int tx, ty;
    const int side = target<I>(G, x, y, tx, ty);
    const double v = side < 0 ? pv.g(I, (long long)ty * G.nx + tx)
                              : (pv.g(opp(I), k) - C.gconst[side][opp(I)]) * C.gsign[side];
    Codec<S>::store(dst + (long long)(9 + I) * G.plane + o, (R)v, C.gscale);
}

template <class S, int NG, int MODE>
__global__ __launch_bounds__(256) void k_unstream(Geom G, Coeffs C, S* __restrict__ dst, const double* pf,
                                                  const double* pg, const double* Tf, double T0) {
    using R = typename Codec<S>::R;
    const long long n = (long long)G.nx * G.ny;
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int x = (int)(k % G.nx), y = (int)(k / G.nx);
    const long long o = (long long)y * G.pitch + x;
    const PreValue<Codec<S>::kDev, NG, MODE> pv{pf, pg, Tf, n, T0, C.varpi, C.tb, C.tgx, C.tgy, C.r0, C.rA, C.rB, G.nx};
    Codec<S>::store(dst + o, (R)pv.f(0, k), C.fscale);
    unstream_f<S, NG, MODE, 1>(dst, G, C, pv, x, y, k, o);
    unstream_f<S, NG, MODE, 2>(dst, G, C, pv, x, y, k, o);
    unstream_f<S, NG, MODE, 3>(dst, G, C, pv, x, y, k, o);
    unstream_f<S, NG, MODE, 4>(dst, G, C, pv, x, y, k, o);
    unstream_f<S, NG, MODE, 5>(dst, G, C, pv, x, y, k, o);
    unstream_f<S, NG, MODE, 6>(dst, G, C, pv, x, y, k, o);
    unstream_f<S, NG, MODE, 7>(dst, G, C, pv, x, y, k, o);
    unstream_f<S, NG, MODE, 8>(dst, G, C, pv, x, y, k, o);
    if constexpr (NG > 0) {
        Codec<S>::store(dst + 9 * G.plane + o, (R)pv.g(0, k), C.gscale);
        unstream_g<S, NG, MODE, 1>(dst, G, C, pv, x, y, k, o);
        unstream_g<S, NG, MODE, 2>(dst, G, C, pv, x, y, k, o);
        unstream_g<S, NG, MODE, 3>(dst, G, C, pv, x, y, k, o);
        unstream_g<S, NG, MODE, 4>(dst, G, C, pv, x, y, k, o);
    }
    if constexpr (NG == 9) {
        unstream_g<S, NG, MODE, 5>(dst, G, C, pv, x, y, k, o);
        unstream_g<S, NG, MODE, 6>(dst, G, C, pv, x, y, k, o);
        unstream_g<S, NG, MODE, 7>(dst, G, C, pv, x, y, k, o);
        unstream_g<S, NG, MODE, 8>(dst, G, C, pv, x, y, k, o);
    }
}

// Temperature at a node from its (pulled or extrapolated) populations.
template <class S, int NG>
__device__ __forceinline__ double node_T(const S* __restrict__ src, const Geom& G, const Coeffs& C, int x, int y) {
    using R = typename Codec<S>::R;
    R f[9], g[gdim(NG)];
    load_node<S, NG>(src, G, C, x, y, f, g);
    return macro_at<S, R, NG>(f, g, C, x, y).T;
}

// Fixed-order block reductions (wave64 shuffles, then LDS in wave order).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

__device__ __forceinline__ void wave_maxloc(double& v, int& i) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_down(v, o, 64);
        const int oi = __shfl_down(i, o, 64);
        if (ov > v || (ov == v && oi < i)) { v = ov; i = oi; }
    }
}

// Link-wise walls: wall half a spacing outside node 1, dT/dn from
// (9 T1 - T2 - 8 Tw) / 3, midpoint mean.  NEE walls (nee = 1): wall through
// node 0, dT/dn from (-3 T0 + 4 T1 - T2) / 2, trapezoidal mean.
// Local Nusselt numbers, one thread per wall node (the wall nodes' depth
// profiles are independent).
template <class S, int NG>
__global__ __launch_bounds__(256) void k_nusselt_local(Geom G, Coeffs C, const S* __restrict__ src, int side,
                                                       double tw, double length, double dT, int nee, double* local) {
    const int count = (side == kLeft || side == kRight) ? G.ny : G.nx;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= count) return;
    const double sign = (side == kLeft || side == kBottom) ? 1.0 : -1.0;
    double t[3];
    for (int d = 0; d < 2 + nee; ++d) {
        int x, y;
        if (side == kLeft) { x = d; y = k; }
        else if (side == kRight) { x = G.nx - 1 - d; y = k; }
        else if (side == kBottom) { x = k; y = d; }
        else { x = k; y = G.ny - 1 - d; }
        t[d] = node_T<S, NG>(src, G, C, x, y);
    }
    const double dtdn = nee ? (-3.0 * t[0] + 4.0 * t[1] - t[2]) / 2.0 : (9.0 * t[0] - t[1] - 8.0 * tw) / 3.0;
    local[k] = -length * (sign * dtdn) / dT;
}

// Mean (midpoint rule, or the trapezoidal rule for walls through the nodes)
// and maximum with its index, one block in a fixed order: thread j sums
// local[j], local[j + 256], ..., then waves, then the block.
__global__ __launch_bounds__(256) void k_nusselt_reduce(const double* __restrict__ local, int count, int nee,
                                                        double* out) {
    __shared__ double s_sum[4], s_max[4];
    __shared__ int s_idx[4];
    double sum = 0.0, best = -DBL_MAX;
    int ibest = 0x7fffffff;
    for (int k = threadIdx.x; k < count; k += blockDim.x) {
        const double nu = local[k];
        sum += (nee && (k == 0 || k == count - 1)) ? 0.5 * nu : nu;
        if (nu > best) { best = nu; ibest = k; }
    }
    sum = wave_sum(sum);
    wave_maxloc(best, ibest);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { s_sum[wave] = sum; s_max[wave] = best; s_idx[wave] = ibest; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0, b = -DBL_MAX;
        int bi = 0x7fffffff;
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) {
            t += s_sum[w];
            if (s_max[w] > b || (s_max[w] == b && s_idx[w] < bi)) { b = s_max[w]; bi = s_idx[w]; }
        }
        out[0] = nee ? t / (count - 1) : t / count;
        out[1] = b;
        out[2] = (double)bi;
    }
}

// Residual of one node against its snapshot (which it then replaces):
// max(|ux - ux'|, |uy - uy'|, |T - T'|), and whether rho, u, T are finite.
template <class S, int NG>
__device__ __forceinline__ void residual_node(const S* __restrict__ src, const Geom& G, const Coeffs& C, int x,
                                              int y, double* snap, bool update_only, double& d,
                                              unsigned long long& bad) {
    using R = typename Codec<S>::R;
    const long long n = (long long)G.nx * G.ny, k = (long long)y * G.nx + x;
    R f[9], g[gdim(NG)];
    load_node<S, NG>(src, G, C, x, y, f, g);
    const Macro m = macro_at<S, R, NG>(f, g, C, x, y);
    const bool fin = isfinite(m.rho) && isfinite(m.ux) && isfinite(m.uy) && isfinite(m.T);
    bad = fin ? 0ull : 1ull;
    d = 0.0;
    if (!update_only && fin)
        d = fmax(fmax(fabs(m.ux - snap[k]), fabs(m.uy - snap[n + k])), fabs(m.T - snap[2 * n + k]));
    snap[k] = m.ux;
    snap[n + k] = m.uy;
    snap[2 * n + k] = m.T;
}

// Block max / sum of (d, bad) in a fixed order (blocks of up to 1024
// threads); lane 0 of wave 0 returns it.
__device__ __forceinline__ void block_maxsum(double& d, unsigned long long& bad) {
    __shared__ double s_max[16];
    __shared__ unsigned long long s_bad[16];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        d = fmax(d, __shfl_down(d, o, 64));
        bad += __shfl_down(bad, o, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) { s_max[wave] = d; s_bad[wave] = bad; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        unsigned long long b = 0;
        const int nw = (blockDim.x + 63) >> 6;
        for (int w = 0; w < nw; ++w) { t = fmax(t, s_max[w]); b += s_bad[w]; }
        d = t;
        bad = b;
    }
}

template <class S, int NG>
__global__ __launch_bounds__(256) void k_residual(Geom G, Coeffs C, const S* __restrict__ src, double* snap,
                                                  int update_only, double* pmax, unsigned long long* pbad) {
    const long long n = (long long)G.nx * G.ny;
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double d = 0.0;
    unsigned long long bad = 0;
    if (k < n) residual_node<S, NG>(src, G, C, (int)(k % G.nx), (int)(k / G.nx), snap, update_only != 0, d, bad);
    block_maxsum(d, bad);
    if (threadIdx.x == 0) {
        pmax[blockIdx.x] = d;
        pbad[blockIdx.x] = bad;
    }
}

// One block of 1024 threads, each with eight partials in flight at a time
// (a 256-thread loop of dependent loads took 22 us for the 16384 partials
// of a 2048^2 lattice).  Maximum and integer sum are exact in any order.
constexpr int kReduceThreads = 1024;
__global__ __launch_bounds__(kReduceThreads) void k_reduce_final(const double* pmax, const unsigned long long* pbad,
                                                                 int nparts, double* out) {
    constexpr int U = 8;
    double d = 0.0;
    unsigned long long b = 0;
    for (int i0 = threadIdx.x; i0 < nparts; i0 += U * kReduceThreads) {
        double v[U];
        unsigned long long c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * kReduceThreads;
            v[u] = i < nparts ? pmax[i] : 0.0;
            c[u] = i < nparts ? pbad[i] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            d = fmax(d, v[u]);
            b += c[u];
        }
    }
    block_maxsum(d, b);
    if (threadIdx.x == 0) {
        out[0] = d;
        out[1] = (double)b;
    }
}

// Residual of every member of a batch: one workgroup per tile, partial
// maxima and non-finite counts per tile, then one workgroup per member
// reduces its contiguous range of tiles (fixed order) into out2[2 m],
// out2[2 m + 1].
template <class S, int NG>
__global__ __launch_bounds__(256) void k_residual_batch(const BatchMember* __restrict__ members,
                                                        const BatchTile* __restrict__ tiles, int parity,
                                                        double* tile_max, unsigned long long* tile_bad) {
    const int ti = blockIdx.x;
    const BatchTile t = tiles[ti];
    const BatchMember& M = members[t.member];
    const S* src = static_cast<const S*>(M.buf[(M.cur0 + parity) & 1]);
    const int x = t.x0 + (int)(threadIdx.x % (unsigned)t.bx);
    const int y = t.y0 + (int)(threadIdx.x / (unsigned)t.bx);
    double d = 0.0;
    unsigned long long bad = 0;
    if (x < M.G.nx && y < M.G.ny) residual_node<S, NG>(src, M.G, M.C, x, y, M.snap, false, d, bad);
    block_maxsum(d, bad);
    if (threadIdx.x == 0) {
        tile_max[ti] = d;
        tile_bad[ti] = bad;
    }
}

__global__ __launch_bounds__(256) void k_reduce_members(const BatchMember* __restrict__ members,
                                                        const double* tile_max, const unsigned long long* tile_bad,
                                                        double* out2) {
    const BatchMember& M = members[blockIdx.x];
    double d = 0.0;
    unsigned long long b = 0;
    for (int i = threadIdx.x; i < M.ntiles; i += blockDim.x) {
        d = fmax(d, tile_max[M.tile0 + i]);
        b += tile_bad[M.tile0 + i];
    }
    block_maxsum(d, b);
    if (threadIdx.x == 0) {
        out2[2 * blockIdx.x] = d;
        out2[2 * blockIdx.x + 1] = (double)b;
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers (internal; the C ABI is in lbm_api.hip).
// ---------------------------------------------------------------------------
static inline int blocks_for(long long n, int bs) { return (int)((n + bs - 1) / bs); }

// Runs the statement with S (storage type) and NG (temperature lattice) bound.
#define LBM_DISPATCH(storage, ng, ...)                                                    \
    switch ((storage) * 16 + (ng)) {                                                      \
        case kF64 * 16 + 0: { using S = double; constexpr int NG = 0; __VA_ARGS__; } break; \
        case kF64 * 16 + 5: { using S = double; constexpr int NG = 5; __VA_ARGS__; } break; \
        case kF64 * 16 + 9: { using S = double; constexpr int NG = 9; __VA_ARGS__; } break; \
        case kF32 * 16 + 0: { using S = float; constexpr int NG = 0; __VA_ARGS__; } break;  \
        case kF32 * 16 + 5: { using S = float; constexpr int NG = 5; __VA_ARGS__; } break;  \
        case kF32 * 16 + 9: { using S = float; constexpr int NG = 9; __VA_ARGS__; } break;  \
        case kF16 * 16 + 0: { using S = __half; constexpr int NG = 0; __VA_ARGS__; } break; \
        case kF16 * 16 + 5: { using S = __half; constexpr int NG = 5; __VA_ARGS__; } break; \
        case kF16 * 16 + 9: { using S = __half; constexpr int NG = 9; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue;                                             \
    }

// The comparison operators (BGK, orthogonal MRT) run one row per thread.
template <class S, int NG, int MODE>
static void sweep_launch(int rows, int coll, dim3 grid, dim3 block, hipStream_t st, const Geom& G,
                         const Coeffs* C, const S* s, S* d, int tiles_x, unsigned bytes, int remap) {
    if (coll == kCollBGK)
        hipLaunchKernelGGL((k_sweep<S, NG, 1, MODE, kCollBGK>), grid, block, 0, st, G, C, s, d, tiles_x, bytes, remap);
    else if (coll == kCollOrtho)
        hipLaunchKernelGGL((k_sweep<S, NG, 1, MODE, kCollOrtho>), grid, block, 0, st, G, C, s, d, tiles_x, bytes,
                           remap);
    else if (rows == 1)
        hipLaunchKernelGGL((k_sweep<S, NG, 1, MODE, kCollMRT>), grid, block, 0, st, G, C, s, d, tiles_x, bytes, remap);
    else
        hipLaunchKernelGGL((k_sweep<S, NG, 2, MODE, kCollMRT>), grid, block, 0, st, G, C, s, d, tiles_x, bytes, remap);
}

template <class S, int NG>
static hipError_t sweep_t(const Launch& L, const Geom& G, const Coeffs& Ch, const Coeffs* C, const void* src,
                          void* dst, hipStream_t st) {
    const int coll = Ch.collision;
    const int rows = coll == kCollMRT ? L.rows : 1;
    if (rows != 1 && rows != 2) return hipErrorInvalidValue;
    if (coll < kCollMRT || coll > kCollOrtho) return hipErrorInvalidValue;
    const int tiles_x = (G.nx + L.bx - 1) / L.bx;
    const int tiles_y = (G.ny + L.by * rows - 1) / (L.by * rows);
    const int nt = tiles_x * tiles_y;
    const S* s = static_cast<const S*>(src);
    S* d = static_cast<S*>(dst);
    const unsigned long long bytes = buffer_bytes<S>(G);
    const dim3 grid(nt), block(L.bx, L.by);
    // strips need a whole number of tiles per XCD in every row
    const int remap = (L.order == kXcdStrips && tiles_x % 8 != 0) ? kXcdBands : L.order;
    if (!L.buffer || bytes >= (1ull << 32))
        sweep_launch<S, NG, kGlobal>(rows, coll, grid, block, st, G, C, s, d, tiles_x, 0u, remap);
    else if (L.keep)
        sweep_launch<S, NG, kBufferKeep>(rows, coll, grid, block, st, G, C, s, d, tiles_x, (unsigned)bytes, remap);
    else
        sweep_launch<S, NG, kBufferNT>(rows, coll, grid, block, st, G, C, s, d, tiles_x, (unsigned)bytes, remap);
    return hipGetLastError();
}


int fuse2_rows(int storage, int ng) {
    LBM_DISPATCH(storage, ng, return Fuse2<S, NG>::TY);
    return 0;
}

template <class S, int NG, int MODE, int COLL>
static void sweep2_launch1(int ntiles, hipStream_t st, const Geom& G, const Coeffs* C, const S* s, S* d, int tiles_x,
                           unsigned bytes, int order) {
    hipLaunchKernelGGL((k_sweep2<S, NG, MODE, COLL>), dim3(ntiles), dim3(Fuse2<S, NG>::NT), 0, st, G, C, s, d, tiles_x,
                       bytes, order);
}

template <class S, int NG, int MODE>
static void sweep2_launch(int coll, int ntiles, hipStream_t st, const Geom& G, const Coeffs* C, const S* s, S* d,
                          int tiles_x, unsigned bytes, int order) {
    if (coll == kCollBGK) sweep2_launch1<S, NG, MODE, kCollBGK>(ntiles, st, G, C, s, d, tiles_x, bytes, order);
    else if (coll == kCollOrtho) sweep2_launch1<S, NG, MODE, kCollOrtho>(ntiles, st, G, C, s, d, tiles_x, bytes, order);
    else sweep2_launch1<S, NG, MODE, kCollMRT>(ntiles, st, G, C, s, d, tiles_x, bytes, order);
}

template <class S, int NG>
static hipError_t sweep2_t(const Launch& L, const Geom& G, const Coeffs& Ch, const Coeffs* C, const void* src,
                           void* dst, hipStream_t st) {
    using F = Fuse2<S, NG>;
    const unsigned long long bytes = buffer_bytes<S>(G);
    const int coll = Ch.collision;
    if (!L.buffer || bytes >= (1ull << 32) || coll < kCollMRT || coll > kCollOrtho) return hipErrorInvalidValue;
    const int tiles_x = (G.nx + F::TX - 1) / F::TX;
    const int tiles_y = (G.ny + F::TY - 1) / F::TY;
    const int order = (L.order == kXcdStrips && tiles_x % 8 != 0) ? kXcdBands : L.order;
    const S* s = static_cast<const S*>(src);
    S* d = static_cast<S*>(dst);
    const int ntiles = tiles_x * tiles_y;
    if (L.keep) sweep2_launch<S, NG, kBufferKeep>(coll, ntiles, st, G, C, s, d, tiles_x, (unsigned)bytes, order);
    else sweep2_launch<S, NG, kBufferNT>(coll, ntiles, st, G, C, s, d, tiles_x, (unsigned)bytes, order);
    return hipGetLastError();
}


// K steps per launch, every collision operator: FP64 and FP32 storage with
// the D2Q5 model or no temperature field, and FP64 storage with the D2Q9
// thermal model.  Not for FP32 D2Q9 thermal: three steps on 32 x 8 tiles
// (two buffers, no spill) were only 1-3% faster than fused pairs at 2048^2
// and 4096^2 and 22% slower at 512^2.  Not for FP16 storage: the kernel is
// generic over the storage (bitwise equal to single steps, tested), but on
// MI355X three steps per launch on 64 x 8 tiles lost to FP16 fused pairs at
// every size (2048^2 D2Q5 45.7 against 33.6 us per step, 4096^2 172
// against 140), the conversions of every value to and from FP16 making the
// longer launch issue-bound.
static constexpr bool fusek_built(int storage, int ng) {
    return ((storage == kF64 || storage == kF32) && (ng == 5 || ng == 0)) || (storage == kF64 && ng == 9);
}

// Runs the statement with S and NG bound for every built multi-step kernel.
#define LBM_DISPATCHK(storage, ng, ...)                                                   \
    switch ((storage) * 16 + (ng)) {                                                      \
        case kF64 * 16 + 0: { using S = double; constexpr int NG = 0; __VA_ARGS__; } break; \
        case kF64 * 16 + 5: { using S = double; constexpr int NG = 5; __VA_ARGS__; } break; \
        case kF64 * 16 + 9: { using S = double; constexpr int NG = 9; __VA_ARGS__; } break; \
        case kF32 * 16 + 0: { using S = float; constexpr int NG = 0; __VA_ARGS__; } break;  \
        case kF32 * 16 + 5: { using S = float; constexpr int NG = 5; __VA_ARGS__; } break;  \
        default: break;                                                                   \
    }

template <class S, int NG>
using FuseKOf = FuseKT<S, NG, fusek_steps<S, NG>()>;

int fusek_tile_rows(int storage, int ng) {
    LBM_DISPATCHK(storage, ng, return FuseKOf<S, NG>::TY);
    return 0;
}

int fusek_tile_cols(int storage, int ng) {
    LBM_DISPATCHK(storage, ng, return FuseKOf<S, NG>::TX);
    return 0;
}

int fusek_launch_steps(int storage, int ng) {
    LBM_DISPATCHK(storage, ng, return fusek_steps<S, NG>());
    return 0;
}

template <class S, int NG, int MODE, int COLL>
static void sweepk_launch1(int ntiles, hipStream_t st, const Geom& G, const Coeffs* C, const S* s, S* d, int tiles_x,
                           unsigned bytes, int order) {
    hipLaunchKernelGGL((k_sweepk<S, NG, fusek_steps<S, NG>(), MODE, COLL>), dim3(ntiles), dim3(FuseKOf<S, NG>::NT),
                       0, st, G, C, s, d, tiles_x, bytes, order);
}

template <class S, int NG>
static hipError_t sweepk_t(const Launch& L, const Geom& G, const Coeffs& Ch, const Coeffs* C, const void* src,
                           void* dst, hipStream_t st) {
    using F = FuseKOf<S, NG>;
    const unsigned long long bytes = buffer_bytes<S>(G);
    const int coll = Ch.collision;
    if (!L.buffer || bytes >= (1ull << 32) || coll < kCollMRT || coll > kCollOrtho) return hipErrorInvalidValue;
    const int tiles_x = (G.nx + F::TX - 1) / F::TX;
    const int tiles_y = (G.ny + F::TY - 1) / F::TY;
    const int order = (L.order == kXcdStrips && tiles_x % 8 != 0) ? kXcdBands : L.order;
    const S* s = static_cast<const S*>(src);
    S* d = static_cast<S*>(dst);
    const int ntiles = tiles_x * tiles_y;
    const unsigned b = (unsigned)bytes;
    if (L.keep) {
        if (coll == kCollBGK) sweepk_launch1<S, NG, kBufferKeep, kCollBGK>(ntiles, st, G, C, s, d, tiles_x, b, order);
        else if (coll == kCollOrtho) sweepk_launch1<S, NG, kBufferKeep, kCollOrtho>(ntiles, st, G, C, s, d, tiles_x, b, order);
        else sweepk_launch1<S, NG, kBufferKeep, kCollMRT>(ntiles, st, G, C, s, d, tiles_x, b, order);
    } else {
        if (coll == kCollBGK) sweepk_launch1<S, NG, kBufferNT, kCollBGK>(ntiles, st, G, C, s, d, tiles_x, b, order);
        else if (coll == kCollOrtho) sweepk_launch1<S, NG, kBufferNT, kCollOrtho>(ntiles, st, G, C, s, d, tiles_x, b, order);
        else sweepk_launch1<S, NG, kBufferNT, kCollMRT>(ntiles, st, G, C, s, d, tiles_x, b, order);
    }
    return hipGetLastError();
}

hipError_t launch_sweepk(int storage, int ng, const Launch& L, const Geom& G, const Coeffs& C, const Coeffs* dC,
                         const void* src, void* dst, hipStream_t st) {
    if (!fusek_built(storage, ng)) return hipErrorInvalidValue;
    LBM_DISPATCHK(storage, ng, return sweepk_t<S, NG>(L, G, C, dC, src, dst, st));
    return hipErrorInvalidValue;
}

hipError_t launch_sweepk_batch(int storage, int ng, bool keep, const BatchMember* members, const BatchTile* tiles,
                               int ntiles, int parity, int order, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    if (!fusek_built(storage, ng)) return hipErrorInvalidValue;
    auto go = [&](auto s, auto n) {
        using S = decltype(s);
        constexpr int NG = decltype(n)::value;
        constexpr int K = fusek_steps<S, NG>();
        if (keep)
            hipLaunchKernelGGL((k_sweepk_batch<S, NG, K, kBufferKeep>), dim3(ntiles), dim3(FuseKOf<S, NG>::NT), 0, st,
                               members, tiles, parity, order);
        else
            hipLaunchKernelGGL((k_sweepk_batch<S, NG, K, kBufferNT>), dim3(ntiles), dim3(FuseKOf<S, NG>::NT), 0, st,
                               members, tiles, parity, order);
    };
    LBM_DISPATCHK(storage, ng, go(S{}, std::integral_constant<int, NG>{}));
    return hipGetLastError();
}

hipError_t launch_sweep2(int storage, int ng, const Launch& L, const Geom& G, const Coeffs& C, const Coeffs* dC,
                         const void* src, void* dst, hipStream_t st) {
    LBM_DISPATCH(storage, ng, { hipError_t e = sweep2_t<S, NG>(L, G, C, dC, src, dst, st); if (e != hipSuccess) return e; });
    return hipSuccess;
}

hipError_t launch_sweep(int storage, int ng, const Launch& L, const Geom& G, const Coeffs& C, const Coeffs* dC,
                        const void* src, void* dst, hipStream_t st) {
    LBM_DISPATCH(storage, ng, { hipError_t e = sweep_t<S, NG>(L, G, C, dC, src, dst, st); if (e != hipSuccess) return e; });
    return hipSuccess;
}

hipError_t launch_sweep_batch(int storage, int ng, bool buffer, bool keep, const BatchMember* members,
                              const BatchTile* tiles, int ntiles, int parity, int order, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    LBM_DISPATCH(storage, ng, {
        if (buffer && keep)
            hipLaunchKernelGGL((k_sweep_batch<S, NG, kBufferKeep>), dim3(ntiles), dim3(256), 0, st, members, tiles, parity,
                               order);
        else if (buffer)
            hipLaunchKernelGGL((k_sweep_batch<S, NG, kBufferNT>), dim3(ntiles), dim3(256), 0, st, members, tiles, parity,
                               order);
        else
            hipLaunchKernelGGL((k_sweep_batch<S, NG, kGlobal>), dim3(ntiles), dim3(256), 0, st, members, tiles, parity,
                               order);
    });
    return hipGetLastError();
}

hipError_t launch_sweep2_batch(int storage, int ng, bool keep, const BatchMember* members, const BatchTile* tiles,
                               int ntiles, int parity, int order, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    LBM_DISPATCH(storage, ng, {
        if (keep)
            hipLaunchKernelGGL((k_sweep2_batch<S, NG, kBufferKeep>), dim3(ntiles), dim3(Fuse2<S, NG>::NT), 0, st,
                               members, tiles, parity, order);
        else
            hipLaunchKernelGGL((k_sweep2_batch<S, NG, kBufferNT>), dim3(ntiles), dim3(Fuse2<S, NG>::NT), 0, st,
                               members, tiles, parity, order);
    });
    return hipGetLastError();
}

hipError_t launch_residual_batch(int storage, int ng, const BatchMember* members, int nmembers,
                                 const BatchTile* tiles, int ntiles, int parity, double* tile_max,
                                 unsigned long long* tile_bad, double* out2, hipStream_t st) {
    if (ntiles <= 0 || nmembers <= 0) return hipSuccess;
    LBM_DISPATCH(storage, ng, hipLaunchKernelGGL((k_residual_batch<S, NG>), dim3(ntiles), dim3(256), 0, st, members,
                                                 tiles, parity, tile_max, tile_bad));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_members, dim3(nmembers), dim3(256), 0, st, members, tile_max, tile_bad, out2);
    return hipGetLastError();
}

hipError_t launch_moments(int storage, int ng, const Geom& G, const Coeffs& C, const void* src, double* rho,
                          double* ux, double* uy, double* T, hipStream_t st) {
    const long long n = (long long)G.nx * G.ny;
    LBM_DISPATCH(storage, ng, hipLaunchKernelGGL((k_moments<S, NG>), dim3(blocks_for(n, 256)), dim3(256), 0, st, G, C,
                                                 static_cast<const S*>(src), rho, ux, uy, T));
    return hipGetLastError();
}

hipError_t launch_gather(int storage, int ng, const Geom& G, const Coeffs& C, const void* src, double* pf,
                         double* pg, double T0, hipStream_t st) {
    const long long n = (long long)G.nx * G.ny;
    LBM_DISPATCH(storage, ng, hipLaunchKernelGGL((k_gather<S, NG>), dim3(blocks_for(n, 256)), dim3(256), 0, st, G, C,
                                                 static_cast<const S*>(src), pf, pg, T0));
    return hipGetLastError();
}

hipError_t launch_unstream(int storage, int ng, const Geom& G, const Coeffs& C, void* dst, const double* pf,
                           const double* pg, const double* Tf, double T0, bool from_temperature, hipStream_t st) {
    const long long n = (long long)G.nx * G.ny;
    if (from_temperature) {
        LBM_DISPATCH(storage, ng, hipLaunchKernelGGL((k_unstream<S, NG, 1>), dim3(blocks_for(n, 256)), dim3(256), 0, st,
                                                     G, C, static_cast<S*>(dst), pf, pg, Tf, T0));
    } else {
        LBM_DISPATCH(storage, ng, hipLaunchKernelGGL((k_unstream<S, NG, 0>), dim3(blocks_for(n, 256)), dim3(256), 0, st,
                                                     G, C, static_cast<S*>(dst), pf, pg, Tf, T0));
    }
    return hipGetLastError();
}

hipError_t launch_nusselt(int storage, int ng, const Geom& G, const Coeffs& C, const void* src, int side, double tw,
                          double length, double dT, int nee, double* local, double* out3, hipStream_t st) {
    const int count = (side == kLeft || side == kRight) ? G.ny : G.nx;
    LBM_DISPATCH(storage, ng, hipLaunchKernelGGL((k_nusselt_local<S, NG>), dim3(blocks_for(count, 256)), dim3(256), 0,
                                                 st, G, C, static_cast<const S*>(src), side, tw, length, dT, nee,
                                                 local));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_nusselt_reduce, dim3(1), dim3(256), 0, st, local, count, nee, out3);
    return hipGetLastError();
}

int residual_parts(const Geom& G) { return blocks_for((long long)G.nx * G.ny, 256); }

hipError_t launch_residual(int storage, int ng, const Geom& G, const Coeffs& C, const void* src, double* snap,
                           bool update_only, double* pmax, unsigned long long* pbad, double* out2, hipStream_t st) {
    const int nb = residual_parts(G);
    LBM_DISPATCH(storage, ng, hipLaunchKernelGGL((k_residual<S, NG>), dim3(nb), dim3(256), 0, st, G, C,
                                                 static_cast<const S*>(src), snap, update_only ? 1 : 0, pmax, pbad));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kReduceThreads), 0, st, pmax, pbad, nb, out2);
    return hipGetLastError();
}

}  // namespace lbm
