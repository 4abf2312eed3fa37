// lbm_internal.hpp -- declarations shared by the kernels and the host runtime.
#pragma once

#include "lbm_device.hpp"

namespace lbm {

enum Storage { kF64 = 0, kF32 = 1, kF16 = 2 };

// Launch shape of the sweep: block of bx x by threads, each thread owning
// `rows` consecutive rows of one column.
struct Launch {
    int bx = 256, by = 1, rows = 1;
    bool buffer = true;  // buffer-resource addressing when the buffer is below 4 GiB
    int order = 1;       // XCD tile order: 0 round robin, 1 bands, 2 strips (lbm_kernels.hip)
    bool keep = false;   // default-policy stores (true) or non-temporal stores (false)
    bool fuse2 = false;  // two time steps per launch where the lattice allows it
    bool fusek = false;  // K time steps per launch where the kernel exists and the lattice allows it
};

// A lattice of a batch as the batched step kernel sees it.
struct BatchMember {
    Geom G;
    Coeffs C;
    void* buf[2];
    unsigned buf_bytes;  // bytes of one population buffer
    int cur0;            // buffer holding the state when the tile table was built
    double* snap;        // residual snapshot (3 * nx * ny), or null
    int tile0, ntiles;   // this member's range of the tile table
};

// One workgroup's work in a batched step: bx x (256 / bx) nodes of member
// `member` starting at (x0, y0).
struct BatchTile {
    int member, x0, y0, bx;
};

inline int storage_bytes(int storage) { return storage == kF64 ? 8 : (storage == kF32 ? 4 : 2); }

// Two time steps per launch (MRT collision, buffers below 4 GiB); rows of
// one fused tile.
hipError_t launch_sweep2(int storage, int ng, const Launch& L, const Geom& G, const Coeffs& C, const Coeffs* dC,
                         const void* src, void* dst, hipStream_t st);
int fuse2_rows(int storage, int ng);
// Tile rows, tile columns and time steps per launch of the multi-step
// kernel, or 0 where none is built.
int fusek_tile_rows(int storage, int ng);
int fusek_tile_cols(int storage, int ng);
int fusek_launch_steps(int storage, int ng);
hipError_t launch_sweepk(int storage, int ng, const Launch& L, const Geom& G, const Coeffs& C, const Coeffs* dC,
                         const void* src, void* dst, hipStream_t st);
hipError_t launch_sweepk_batch(int storage, int ng, bool keep, const BatchMember* members, const BatchTile* tiles,
                               int ntiles, int parity, int order, hipStream_t st);
// Fused pairs of steps for a batch (buffer addressing; keep: default-policy stores).
// order: XCD order of the tile table (0 round robin, 1 bands).
hipError_t launch_sweep2_batch(int storage, int ng, bool keep, const BatchMember* members, const BatchTile* tiles,
                               int ntiles, int parity, int order, hipStream_t st);
// C: the host copy (launch decisions); dC: the same constants in device
// memory (read by the kernels).
hipError_t launch_sweep(int storage, int ng, const Launch& L, const Geom& G, const Coeffs& C, const Coeffs* dC,
                        const void* src, void* dst, hipStream_t st);
// keep: default-policy stores (the batch's state fits the last-level cache).
hipError_t launch_sweep_batch(int storage, int ng, bool buffer, bool keep, const BatchMember* members,
                              const BatchTile* tiles, int ntiles, int parity, int order, hipStream_t st);
hipError_t launch_residual_batch(int storage, int ng, const BatchMember* members, int nmembers, const BatchTile* tiles,
                                 int ntiles, int parity, double* tile_max, unsigned long long* tile_bad,
                                 double* out2, hipStream_t st);
hipError_t launch_moments(int storage, int ng, const Geom& G, const Coeffs& C, const void* src, double* rho,
                          double* ux, double* uy, double* T, hipStream_t st);
hipError_t launch_gather(int storage, int ng, const Geom& G, const Coeffs& C, const void* src, double* pf,
                         double* pg, double T0, hipStream_t st);
hipError_t launch_unstream(int storage, int ng, const Geom& G, const Coeffs& C, void* dst, const double* pf,
                           const double* pg, const double* Tf, double T0, bool from_temperature,
                           hipStream_t st);
hipError_t launch_nusselt(int storage, int ng, const Geom& G, const Coeffs& C, const void* src, int side,
                          double tw, double length, double dT, int nee, double* local, double* out3,
                          hipStream_t st);
int residual_parts(const Geom& G);
hipError_t launch_residual(int storage, int ng, const Geom& G, const Coeffs& C, const void* src, double* snap,
                           bool update_only, double* pmax, unsigned long long* pbad, double* out2,
                           hipStream_t st);

}  // namespace lbm
