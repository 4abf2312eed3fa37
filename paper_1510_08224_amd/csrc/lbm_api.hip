// lbm_api.hip -- host runtime behind include/lbm.h: solver lifetime,
// parameter validation and derivation (Eqs. 20, 29, 40), device memory,
// launches on the solver's stream, and readouts.
#include "lbm_internal.hpp"
#include "lbm.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace lbm;

struct lbm_solver {
    int nx = 0, ny = 0, storage = 0;
    int model = LBM_MODEL_D2Q5, ng = 5;  // thermal model and its population count
    Geom G{};
    Coeffs C{};
    Coeffs* d_coeffs = nullptr;  // device copy of C, read by the step kernels
    Launch L{};
    size_t buf_bytes = 0;        // bytes of one population buffer (9 + ng planes)
    void* base = nullptr;        // both buffers, contiguous
    bool own_base = false;
    void* buf[2] = {nullptr, nullptr};
    int cur = 0;                 // buffer holding the state of time t
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = -1;             // HIP device current at create
    bool params_set = false;
    lbm_params params{};
    double s_nu = 0, zeta_alpha = 0, gbeta = 0, T0 = 0, length = 0, dT = 0;
    int64_t t = 0;
    // lazily allocated device scratch
    double* snap = nullptr;      // 3 * nx * ny: residual snapshot (ux, uy, T)
    bool snap_valid = false;
    double* rpart = nullptr;     // residual partial maxima
    unsigned long long* rbad = nullptr;
    double* fields = nullptr;    // 4 * nx * ny: host-bound moments staging
    double* small = nullptr;     // device outputs of reductions (8 doubles)
    double* nu_local = nullptr;  // max(nx, ny)
    double* host_small = nullptr;  // pinned host copy of `small`
    // Captured graphs of graph_steps sweeps (an even count), one per
    // starting buffer; rebuilt after any change of parameters or launch.
    int graph_steps = 0;
    int64_t graph_launches = 0;  // launches in one captured graph (fused pairs count once)
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
    lbm_batch* batch = nullptr;  // batch this solver belongs to, if any
    // Tracing (environment variable LBM_PROFILE set and not "0" at create):
    // HIP events bracket each lbm_step call on the solver's stream; pairs
    // are folded into the totals once complete, and lbm_destroy prints a
    // one-line JSON summary to stderr.
    bool prof = false;
    std::vector<hipEvent_t> prof_ev;   // pending start, stop, start, stop, ...
    double prof_ms = 0.0;
    int64_t prof_calls = 0, prof_steps = 0, prof_launches = 0;
    mutable std::string err;  // last error; const readouts report theirs too
};

struct lbm_batch {
    int storage = 0;
    int ng = -1;                      // thermal populations of the members (set by the first)
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<lbm_solver*> slots;   // nullptr = free slot
    bool dirty = true;                // tile table must be rebuilt
    int parity = 0;                   // steps since the table was built, mod 2
    bool buffer = true;
    BatchMember* d_members = nullptr;
    BatchTile* d_tiles = nullptr;
    size_t cap_members = 0, cap_tiles = 0;
    int ntiles = 0;
    // Fused pairs of steps: the policy asked for (LBM_POLICY_DEFAULT, 0 or
    // LBM_POLICY_FUSE2), whether the current members use them, whether the
    // stores of either kernel keep the default cache policy (all members'
    // buffers within the 256 MB last-level cache), and the fused tile table.
    int policy = LBM_POLICY_DEFAULT;
    bool fuse = false, keep = false;
    // Tuning of the launches (lbm_batch_set_tuning): XCD order of the tile
    // tables (-1: bands; 0 round robin, 1 bands), stores (-1: the footprint
    // rule; 0 non-temporal, 1 kept), tile-table order of the members (0 as
    // added, 1 largest first); `order` is the order in effect.
    int tune_order = -1, tune_keep = -1, tune_sort = 0;
    int order = 1;
    BatchTile* d_ftiles = nullptr;
    size_t cap_ftiles = 0;
    int nftiles = 0;
    // K steps per launch (LBM_POLICY_FUSEK): whether the current members
    // use them, and their tile table (tiles of the multi-step kernel).
    bool fusek = false;
    BatchTile* d_fktiles = nullptr;
    size_t cap_fktiles = 0;
    int nfktiles = 0;
    std::vector<int> member_slot;     // tile-table member index -> slot
    double* d_tile_max = nullptr;     // batched residual scratch
    unsigned long long* d_tile_bad = nullptr;
    double* d_rout = nullptr;
    double* h_rout = nullptr;
    size_t cap_rtiles = 0, cap_rout = 0;
    int graph_steps = 0;
    int64_t graph_launches = 0;       // launches in one captured graph
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
    std::string err;
};

static void batch_invalidate(lbm_batch* b);

static thread_local std::string g_create_error;

static int fail(const lbm_solver* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    else g_create_error = msg;
    return code;
}

static int hip_fail(lbm_solver* h, hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
    return fail(h, LBM_ERR_DEVICE, m);
}

#define LBM_HIP(h, call, what)                                  \
    do {                                                        \
        hipError_t _e = (call);                                 \
        if (_e != hipSuccess) return hip_fail((h), _e, (what)); \
    } while (0)

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Temperature populations per node of a thermal model.
static int model_ng(int model) { return model == LBM_MODEL_D2Q5 ? 5 : (model == LBM_MODEL_D2Q9T ? 9 : 0); }
static bool model_ok(int model) { return model >= LBM_MODEL_D2Q5 && model <= LBM_MODEL_ISOTHERMAL; }

// Rows interleaved by population: row y of the buffer holds row y of each of
// the 9 + NG populations in turn, each padded to whole 256-byte segments
// (`plane` elements); a row of nodes takes pitch = (9 + NG) * plane
// elements, and the buffer ny rows, rounded up to 4 KiB.
// False if a row of nodes would take 2^31 elements or more (the kernels
// hold the row pitch in 32 bits).
static bool layout(int nx, int ny, int storage, int ng, int* pitch, long long* plane, size_t* buf_bytes) {
    const size_t b = storage_bytes(storage);
    const size_t p = align_up((size_t)nx, 256 / b);
    const size_t row = (size_t)(9 + ng) * p;
    *pitch = row < (1ull << 31) ? (int)row : 0;
    *plane = (long long)p;
    *buf_bytes = align_up(row * (size_t)ny * b, 4096);
    return row < (1ull << 31);
}

extern "C" {

void lbm_params_default(lbm_params* p) {
    if (!p) return;
    memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(lbm_params);
    p->pr = 0.71;
    p->t_hot = 1.0;
    p->t_cold = 0.0;
    p->s_e = 1.6;
    p->s_q = 1.2;
    p->s_eps = 1.8;
    p->zeta_e = 1.9;
    p->zeta_nu = 1.9;
    p->zeta_q = 1.9;
    p->zeta_eps = 1.9;
    p->varpi = 0.5;
    p->theta = 1.0;
    for (int s = 0; s < 4; ++s) p->bc_flow[s] = LBM_BC_WALL;
    p->bc_temp[LBM_LEFT] = LBM_T_DIRICHLET;
    p->bc_temp[LBM_RIGHT] = LBM_T_DIRICHLET;
    p->bc_temp[LBM_BOTTOM] = LBM_T_ADIABATIC;
    p->bc_temp[LBM_TOP] = LBM_T_ADIABATIC;
    p->wall_T[LBM_LEFT] = 1.0;
    p->wall_T[LBM_RIGHT] = 0.0;
}

// Sec. 3.2: Re = L u / nu, nu = (1/s_nu - 1/2) / 3.
int lbm_rate_for_reynolds(double re, double length, double u, double* s_nu) {
    if (!s_nu || !(re > 0.0) || !(length > 0.0) || !(u > 0.0) || !isfinite(re) || !isfinite(length) || !isfinite(u))
        return fail(nullptr, LBM_ERR_ARG, "lbm_rate_for_reynolds: Re, length and u must be finite and positive");
    *s_nu = 1.0 / (0.5 + 3.0 * length * u / re);
    return LBM_OK;
}

int32_t lbm_abi_version(void) { return LBM_ABI_VERSION; }

const char* lbm_build_info(void) {
    return "lbm non-orthogonal MRT: D2Q9 flow with D2Q5, D2Q9 or no temperature lattice; HIP gfx950; "
           "storage f64/f32/f16";
}

int lbm_required_bytes(int32_t nx, int32_t ny, int32_t storage, int32_t model, uint64_t* bytes) {
    if (!bytes || nx < 1 || ny < 1 || storage < LBM_F64 || storage > LBM_F16 || !model_ok(model))
        return fail(nullptr, LBM_ERR_ARG, "lbm_required_bytes: bad size, storage, model or NULL output");
    if ((long long)nx * ny > (1ll << 31))
        return fail(nullptr, LBM_ERR_ARG, "lbm_required_bytes: more than 2^31 nodes");
    int pitch;
    long long plane;
    size_t bb;
    if (!layout(nx, ny, storage, model_ng(model), &pitch, &plane, &bb))
        return fail(nullptr, LBM_ERR_ARG, "lbm_required_bytes: a row of nodes would take 2^31 elements or more");
    *bytes = 2 * (uint64_t)bb;
    return LBM_OK;
}

// Memory policy from the footprint of both population buffers, measured on
// MI355X (512^2 to 4096^2 lattices, every model and storage,
// `tuning.py`): when both fit the 256 MB last-level cache, stores keep their
// lines there; above it non-temporal stores win.  K = 4 steps per launch
// (LBM_POLICY_FUSEK; FP64 and FP32 storage, the D2Q5 model or no
// temperature field) win for FP64 at every size (D2Q5 over the best fused
// pair: 512^2 +16%, 1024^2 +15% with kept stores, 2048^2 +52%, 4096^2
// +55%; the flow alone +9% to +55%, within 4% of the pair at 512^2) and for
// FP32 beyond the last-level cache (2048^2 and 4096^2: D2Q5 +10% and +15%, the
// flow alone +23% and +29%) and up to 96 MiB (512^2: D2Q5 +11%, the flow
// alone +15%; 1024^2 flow alone, 75 MB, +5%), but not for the 117 MB FP32
// D2Q5 state of 1024^2 (the pair with kept stores 10% faster); they
// need XCD bands (strips or round robin took 8-59% longer).  The FP64 D2Q9
// thermal model takes three steps per launch on 32 x 8 tiles (per step:
// 512^2 -3%, 1024^2 -16%, 2048^2 and 4096^2 -21% against the best pair).  Fused pairs
// (LBM_POLICY_FUSE2) win over single steps for every storage and model at
// every size (FP16 included: 2048^2 D2Q5, a 235 MB state, +13% over kept
// single stores; the flow alone +9% to +22%), with bands, or strips (with
// a multiple of 8 tiles per row) once one row of fused tiles exceeds 3 MiB
// or an FP64 lattice is 48 or more tiles wide; pairs stay on for
// remainders and wherever K-step launches do not apply.
static void default_policy(lbm_solver* h) {
    const double ws = 2.0 * (double)h->buf_bytes, mib = 1024.0 * 1024.0;
    h->L.keep = ws <= 256.0 * mib;
    h->L.fuse2 = true;
    const bool f32k = ws > 256.0 * mib || ws <= 96.0 * mib;
    h->L.fusek = fusek_launch_steps(h->storage, h->ng) > 0 &&
                 (h->storage == LBM_F64 || (h->storage == LBM_F32 && f32k));
    if (h->L.fusek) {
        h->L.order = 1;
    } else {
        // Bands keep the halo rows a fused tile shares with the tile row
        // below in the XCD's 4 MB L2 while one row of tiles (tile and halo,
        // every plane) fits there; past that, strips of 8 tiles per XCD do.
        // FP64 lattices 48 or more tiles wide take strips at any row size
        // (3072^2 and 4096^2, every model: +2.3 to +5.4%; at 2048^2 bands
        // win by up to 7%); FP32 keeps bands below 3 MiB per row.
        const int ty = fuse2_rows(h->storage, h->ng);
        const int tiles_x = (h->nx + 63) / 64;
        const double row = (double)tiles_x * 66.0 * (ty + 2) * (9 + h->ng) * storage_bytes(h->storage);
        const bool strips = row > 3.0 * mib || (h->storage == LBM_F64 && tiles_x >= 48);
        h->L.order = (tiles_x % 8 == 0 && strips) ? 2 : 1;
    }
}

static void default_launch(lbm_solver* h) {
    // Measured on MI355X (1024^2 to 4096^2, every model and storage): 64 x 4
    // blocks for FP64 storage and for any state of up to about 320 MB, full
    // 256-wide rows for larger FP32/FP16 states; one row per thread (more
    // rows per thread cost occupancy and lose bandwidth).
    const double ws = 2.0 * (double)h->buf_bytes;
    int bx = (h->storage == LBM_F64 || ws <= 320.0 * 1024 * 1024) ? 64 : 256;
    while (bx > 64 && bx / 2 >= h->nx) bx /= 2;
    h->L.bx = bx;
    h->L.by = 256 / bx;
    h->L.rows = 1;
    default_policy(h);
    // Small lattices finish a sweep in a few microseconds, less than a
    // kernel launch costs: replay captured graphs of many sweeps instead.
    h->graph_steps = ((long long)h->nx * h->ny <= (1ll << 18)) ? 64 : 0;
}

static void drop_graphs(lbm_solver* h) {
    for (int k = 0; k < 2; ++k) {
        if (h->graph_exec[k]) (void)hipGraphExecDestroy(h->graph_exec[k]);
        h->graph_exec[k] = nullptr;
    }
}

static int create_common(lbm_solver** out, int32_t nx, int32_t ny, int32_t storage, int32_t model,
                         void* dev_buf, uint64_t bytes, void* stream) {
    if (!out) return fail(nullptr, LBM_ERR_ARG, "lbm_create: NULL output handle");
    *out = nullptr;
    if (nx < 1 || ny < 1) return fail(nullptr, LBM_ERR_ARG, "lbm_create: nx and ny must be >= 1");
    if ((long long)nx * ny > (1ll << 31))
        return fail(nullptr, LBM_ERR_ARG, "lbm_create: more than 2^31 nodes");
    if (storage < LBM_F64 || storage > LBM_F16)
        return fail(nullptr, LBM_ERR_ARG, "lbm_create: storage must be LBM_F64, LBM_F32 or LBM_F16");
    if (!model_ok(model)) return fail(nullptr, LBM_ERR_ARG, "lbm_create: unknown thermal model");
    lbm_solver* h = new (std::nothrow) lbm_solver();
    if (!h) return fail(nullptr, LBM_ERR_NOMEM, "lbm_create: host allocation failed");
    h->nx = nx;
    h->ny = ny;
    h->storage = storage;
    h->model = model;
    if (hipGetDevice(&h->device) != hipSuccess) h->device = -1;
    h->ng = model_ng(model);
    if (!layout(nx, ny, storage, h->ng, &h->G.pitch, &h->G.plane, &h->buf_bytes)) {
        delete h;
        return fail(nullptr, LBM_ERR_ARG, "lbm_create: a row of nodes would take 2^31 elements or more");
    }
    h->G.nx = nx;
    h->G.ny = ny;
    const uint64_t need = 2 * (uint64_t)h->buf_bytes;
    if (dev_buf) {
        if (bytes < need) {
            delete h;
            return fail(nullptr, LBM_ERR_NOMEM, "lbm_create_ext: buffer smaller than lbm_required_bytes()");
        }
        if (((uintptr_t)dev_buf & 255) != 0) {
            delete h;
            return fail(nullptr, LBM_ERR_ARG, "lbm_create_ext: buffer not 256-byte aligned");
        }
        h->base = dev_buf;
        h->own_base = false;
    } else {
        hipError_t e = hipMalloc(&h->base, need);
        if (e != hipSuccess) {
            delete h;
            return fail(nullptr, LBM_ERR_NOMEM, std::string("lbm_create: hipMalloc failed: ") + hipGetErrorString(e));
        }
        h->own_base = true;
    }
    h->buf[0] = h->base;
    h->buf[1] = static_cast<char*>(h->base) + h->buf_bytes;
    if (stream) {
        h->stream = static_cast<hipStream_t>(stream);
    } else {
        hipError_t e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            if (h->own_base) (void)hipFree(h->base);
            delete h;
            return fail(nullptr, LBM_ERR_DEVICE, std::string("lbm_create: stream creation failed: ") + hipGetErrorString(e));
        }
        h->own_stream = true;
    }
    hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&h->host_small), 8 * sizeof(double), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&h->small), 8 * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&h->d_coeffs), sizeof(Coeffs));
    if (e != hipSuccess) {
        lbm_destroy(h);
        return fail(nullptr, LBM_ERR_NOMEM, "lbm_create: small buffers");
    }
    default_launch(h);
    const char* pe = getenv("LBM_PROFILE");
    h->prof = pe && *pe && strcmp(pe, "0") != 0;
    *out = h;
    return LBM_OK;
}

int lbm_create(lbm_solver** out, int32_t nx, int32_t ny, int32_t storage, int32_t model, void* hip_stream) {
    return create_common(out, nx, ny, storage, model, nullptr, 0, hip_stream);
}

int lbm_create_ext(lbm_solver** out, int32_t nx, int32_t ny, int32_t storage, int32_t model,
                   void* device_buffer, uint64_t bytes, void* hip_stream) {
    if (!device_buffer) return fail(nullptr, LBM_ERR_ARG, "lbm_create_ext: NULL device buffer");
    return create_common(out, nx, ny, storage, model, device_buffer, bytes, hip_stream);
}

int32_t lbm_model_of(const lbm_solver* h) { return h ? h->model : -1; }

// Fold completed event pairs into the totals (all of them: wait for each).
static void prof_drain(lbm_solver* h, bool all) {
    size_t k = 0;
    for (; k + 1 < h->prof_ev.size(); k += 2) {
        hipEvent_t a = h->prof_ev[k], b = h->prof_ev[k + 1];
        if (all) (void)hipEventSynchronize(b);
        else if (hipEventQuery(b) != hipSuccess) break;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, a, b) == hipSuccess) h->prof_ms += ms;
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    h->prof_ev.erase(h->prof_ev.begin(), h->prof_ev.begin() + (long)k);
}

static void prof_report(lbm_solver* h) {
    prof_drain(h, true);
    if (!h->prof_calls) return;
    static const char* names[] = {"f64", "f32", "f16"};
    const double mlups = h->prof_ms > 0.0 ? (double)h->nx * h->ny * h->prof_steps / (h->prof_ms * 1e3) : 0.0;
    fprintf(stderr,
            "{\"lbm_profile\": {\"nx\": %d, \"ny\": %d, \"storage\": \"%s\", \"model\": %d, \"calls\": %lld, "
            "\"steps\": %lld, \"launches\": %lld, \"gpu_ms\": %.3f, \"mlups\": %.1f}}\n",
            h->nx, h->ny, names[h->storage], h->model, (long long)h->prof_calls, (long long)h->prof_steps,
            (long long)h->prof_launches, h->prof_ms, mlups);
}

void lbm_destroy(lbm_solver* h) {
    if (!h) return;
    if (h->batch) {
        for (auto& m : h->batch->slots)
            if (m == h) m = nullptr;
        batch_invalidate(h->batch);
        h->batch = nullptr;
    }
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->prof) prof_report(h);
    drop_graphs(h);
    if (h->own_base && h->base) (void)hipFree(h->base);
    if (h->snap) (void)hipFree(h->snap);
    if (h->rpart) (void)hipFree(h->rpart);
    if (h->rbad) (void)hipFree(h->rbad);
    if (h->fields) (void)hipFree(h->fields);
    if (h->small) (void)hipFree(h->small);
    if (h->d_coeffs) (void)hipFree(h->d_coeffs);
    if (h->nu_local) (void)hipFree(h->nu_local);
    if (h->host_small) (void)hipHostFree(h->host_small);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

const char* lbm_last_error(const lbm_solver* h) {
    return h ? h->err.c_str() : g_create_error.c_str();
}

void* lbm_stream(const lbm_solver* h) { return h ? static_cast<void*>(h->stream) : nullptr; }
int32_t lbm_storage_of(const lbm_solver* h) { return h ? h->storage : -1; }

static bool rate_ok(double s) { return isfinite(s) && s > 0.0 && s < 2.0; }

// D2Q9 weights (after Eq. 22) for the moving-wall term.
static const double kW9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

// The relaxation constants in the arithmetic type T, each rounded as a
// kernel colliding in T would round it: the double converted to T, then one
// operation in T.
extern "C++" template <class T>
static void fill_rates(Rates<T>& K, const Coeffs& C) {
    K.s3 = (T)C.s3;
    K.s4 = (T)C.s4;
    K.s6 = (T)C.s6;
    K.s8 = (T)C.s8;
    K.h3 = (T)1 - (T)0.5 * K.s3;
    K.h4 = (T)1 - (T)0.5 * K.s4;
    K.h6 = (T)1 - (T)0.5 * K.s6;
    K.h8 = (T)1 - (T)0.5 * K.s8;
    K.z1 = (T)C.z1;
    K.z3 = (T)C.z3;
    K.z4 = (T)C.z4;
    K.z6 = (T)C.z6;
    K.z8 = (T)C.z8;
    K.varpi = (T)C.varpi;
    K.one_m_varpi = (T)1 - K.varpi;
    K.theta = (T)C.theta;
}

static int derive(lbm_solver* h, const lbm_params* p) {
    if (p->collision < LBM_COLLISION_MRT || p->collision > LBM_COLLISION_ORTHO_MRT)
        return fail(h, LBM_ERR_ARG, "lbm_set_params: unknown collision operator");
    if (p->collision != LBM_COLLISION_MRT && h->batch)
        return fail(h, LBM_ERR_UNSUPPORTED, "lbm_set_params: batch members use the MRT collision");
    int nee = 0, linkwise = 0;
    for (int s = 0; s < 4; ++s) {
        if (p->bc_flow[s] < LBM_BC_PERIODIC || p->bc_flow[s] > LBM_BC_NEE)
            return fail(h, LBM_ERR_ARG, "lbm_set_params: unknown bc_flow code");
        if (p->bc_temp[s] < LBM_T_PERIODIC || p->bc_temp[s] > LBM_T_NEE_ADIABATIC)
            return fail(h, LBM_ERR_ARG, "lbm_set_params: unknown bc_temp code");
        const bool fn = p->bc_flow[s] == LBM_BC_NEE;
        const bool tn = p->bc_temp[s] == LBM_T_NEE_DIRICHLET || p->bc_temp[s] == LBM_T_NEE_ADIABATIC;
        if (fn != tn)
            return fail(h, LBM_ERR_ARG, "lbm_set_params: an NEE flow wall needs an NEE temperature wall and vice versa");
        nee += fn;
        linkwise += p->bc_flow[s] == LBM_BC_WALL;
    }
    if (nee && linkwise)
        return fail(h, LBM_ERR_ARG, "lbm_set_params: NEE and link-wise walls cannot be mixed on one lattice");
    if ((p->bc_flow[LBM_LEFT] == LBM_BC_NEE && h->nx < 3) || (p->bc_flow[LBM_BOTTOM] == LBM_BC_NEE && h->ny < 3))
        return fail(h, LBM_ERR_ARG, "lbm_set_params: NEE walls need at least 3 nodes across");
    for (int a = 0; a < 2; ++a) {
        const int s0 = 2 * a, s1 = 2 * a + 1;
        const bool f0 = p->bc_flow[s0] == LBM_BC_PERIODIC, f1 = p->bc_flow[s1] == LBM_BC_PERIODIC;
        const bool t0 = p->bc_temp[s0] == LBM_T_PERIODIC, t1 = p->bc_temp[s1] == LBM_T_PERIODIC;
        if (f0 != f1 || t0 != t1 || f0 != t0)
            return fail(h, LBM_ERR_ARG, "lbm_set_params: an axis must be periodic on both sides, for flow and temperature, or on neither");
    }
    if (!(isfinite(p->varpi) && p->varpi > 0.0 && p->varpi < 1.0))
        return fail(h, LBM_ERR_ARG, "lbm_set_params: varpi must lie in (0, 1)");
    if (!isfinite(p->t_hot) || !isfinite(p->t_cold) || !isfinite(p->ax) || !isfinite(p->ay))
        return fail(h, LBM_ERR_ARG, "lbm_set_params: non-finite temperature or force");
    for (int s = 0; s < 4; ++s)
        if (!isfinite(p->wall_T[s]) || !isfinite(p->wall_u[s][0]) || !isfinite(p->wall_u[s][1]))
            return fail(h, LBM_ERR_ARG, "lbm_set_params: non-finite wall value");
    // default L: the distance between the bottom and top walls
    const bool q9 = h->ng == 9, iso = h->ng == 0;
    if (q9 && !(p->theta == 0.0 || p->theta == 1.0))
        return fail(h, LBM_ERR_ARG, "lbm_set_params: theta must be 0 or 1 (Eq. 31)");
    const double length = p->length > 0 ? p->length
                                        : (p->bc_flow[LBM_BOTTOM] == LBM_BC_NEE ? (double)(h->ny - 1) : (double)h->ny);
    const double dT = p->t_hot - p->t_cold;
    // c_sT^2 = varpi / 2 for D2Q5 (Sec. 2.2); c_s^2 = 1/3 for D2Q9 (after Eq. 32)
    const double cs2 = 1.0 / 3.0, csT2 = q9 ? cs2 : p->varpi / 2.0;
    double s_nu = p->s_nu, z_a = p->zeta_alpha;
    if (!(s_nu > 0)) {
        if (!(p->u_c > 0 && p->ra > 0 && p->pr > 0))
            return fail(h, LBM_ERR_ARG, "lbm_set_params: s_nu needs ra, pr and u_c > 0 (Eq. 40) or an explicit value");
        const double ma = sqrt(3.0) * p->u_c;
        s_nu = 1.0 / (0.5 + ma * length * sqrt(3.0 * p->pr) / sqrt(p->ra));
    }
    if (!(z_a > 0)) {
        if (!(p->pr > 0)) return fail(h, LBM_ERR_ARG, "lbm_set_params: zeta_alpha needs pr > 0 (Eq. 40) or an explicit value");
        z_a = 1.0 / (0.5 + cs2 * (1.0 / s_nu - 0.5) / (csT2 * p->pr));
    }
    const double rates[9] = {p->s_e, s_nu, p->s_q, p->s_eps, z_a, p->zeta_e, p->zeta_nu,
                             q9 ? p->zeta_q : 1.0, q9 ? p->zeta_eps : 1.0};
    for (double r : rates)
        if (!rate_ok(r)) return fail(h, LBM_ERR_ARG, "lbm_set_params: every relaxation rate must lie in (0, 2)");
    const double gbeta = (!iso && p->u_c > 0 && dT != 0) ? p->u_c * p->u_c / (dT * length) : 0.0;
    const double T0 = 0.5 * (p->t_hot + p->t_cold);
    const bool dev = h->storage != LBM_F64;

    Coeffs C{};
    C.s3 = p->s_e;
    C.s4 = s_nu;
    C.s6 = p->s_q;
    C.s8 = p->s_eps;
    C.z1 = z_a;
    C.z3 = p->zeta_e;
    C.z4 = p->zeta_nu;
    C.z6 = q9 ? p->zeta_q : 1.0;
    C.z8 = q9 ? p->zeta_eps : 1.0;
    C.theta = q9 ? p->theta : 0.0;
    C.T0 = T0;
    C.varpi = p->varpi;
    C.gbeta = gbeta;
    C.ax = p->ax;
    C.ay = p->ay;
    C.tshift = dev ? 0.0 : -T0;
    C.toff = dev ? T0 : 0.0;
    // FP16 reference temperature: the linear conduction profile between the
    // two link-wise Dirichlet walls of one axis (walls half a spacing
    // outside the first and last nodes), when the other axis has no
    // Dirichlet wall and no wall is NEE; tau(p) = T_w0 - T0 + tg (p + 1/2)
    // along that axis, tg = (T_w1 - T_w0) / n.
    C.tb = C.tgx = C.tgy = 0.0;
    for (int i = 0; i < 9; ++i) C.gdc[i] = 0.0f;
    if (h->storage == LBM_F16 && !iso && !nee) {
        const bool dx = p->bc_temp[LBM_LEFT] == LBM_T_DIRICHLET && p->bc_temp[LBM_RIGHT] == LBM_T_DIRICHLET;
        const bool dy = p->bc_temp[LBM_BOTTOM] == LBM_T_DIRICHLET && p->bc_temp[LBM_TOP] == LBM_T_DIRICHLET;
        const bool ax = p->bc_temp[LBM_LEFT] == LBM_T_DIRICHLET || p->bc_temp[LBM_RIGHT] == LBM_T_DIRICHLET;
        const bool ay = p->bc_temp[LBM_BOTTOM] == LBM_T_DIRICHLET || p->bc_temp[LBM_TOP] == LBM_T_DIRICHLET;
        if (dx && !ay) {
            C.tgx = (p->wall_T[LBM_RIGHT] - p->wall_T[LBM_LEFT]) / (double)h->nx;
            C.tb = p->wall_T[LBM_LEFT] - T0 + 0.5 * C.tgx;
        } else if (dy && !ax) {
            C.tgy = (p->wall_T[LBM_TOP] - p->wall_T[LBM_BOTTOM]) / (double)h->ny;
            C.tb = p->wall_T[LBM_BOTTOM] - T0 + 0.5 * C.tgy;
        }
        for (int i = 0; i < 9; ++i) {
            const double ci = q9 ? kW9[i] : (i == 0 ? 1.0 - p->varpi : 0.25 * p->varpi);
            C.gdc[i] = (float)(ci * (C.tgx * ex(i) + C.tgy * ey(i)));
        }
    }
    // FP16, x-periodic, temperature reference along y: the flow populations
    // are kept relative to the hydrostatic density of that reference,
    // rho_ref(y) = r0 + rA y + rB y^2 with 1/3 d rho_ref / dy = a_y + g beta
    // tau(y) (Eq. 4 at rest), r0 making its mean over the rows zero.
    C.r0 = C.rA = C.rB = 0.0;
    C.frA = C.frB = 0.0f;
    if (h->storage == LBM_F16 && C.tgy != 0.0 && p->bc_flow[LBM_LEFT] == LBM_BC_PERIODIC) {
        C.rA = 3.0 * (p->ay + gbeta * C.tb);
        C.rB = 1.5 * gbeta * C.tgy;
        double m1 = 0.0, m2 = 0.0;
        for (int y = 0; y < h->ny; ++y) {
            m1 += (double)y;
            m2 += (double)y * (double)y;
        }
        C.r0 = -(C.rA * m1 + C.rB * m2) / (double)h->ny;
        C.frA = (float)C.rA;
        C.frB = (float)C.rB;
    }
    for (int s = 0; s < 4; ++s) {
        for (int i = 0; i < 9; ++i) {
            const double eu = ex(i) * p->wall_u[s][0] + ey(i) * p->wall_u[s][1];
            C.bbf[s][i] = p->bc_flow[s] == LBM_BC_WALL ? 6.0 * kW9[i] * eu : 0.0;
            // a density reference: the stored opposite population is
            // relative to the reference one row beyond the wall
            if (p->bc_flow[s] == LBM_BC_WALL && s == LBM_BOTTOM && ey(i) == 1)
                C.bbf[s][i] += kW9[i] * (-C.rA + C.rB);
            if (p->bc_flow[s] == LBM_BC_WALL && s == LBM_TOP && ey(i) == -1)
                C.bbf[s][i] += kW9[i] * (C.rA + C.rB * (2.0 * h->ny - 1.0));
        }
        // anti-bounce-back: twice the even part of g^eq at the wall (Eq. 30:
        // varpi T_w / 4 per link; Eq. 31: w_i T_w [1 + theta (4.5 (e.u_w)^2 - 1.5 u_w^2)]),
        // minus twice the stored rest part for deviation storage
        const bool dir = p->bc_temp[s] == LBM_T_DIRICHLET;
        C.gsign[s] = dir ? -1.0 : 1.0;
        // With an FP16 reference temperature the stored opposite population
        // is relative to the reference of the ghost node one spacing beyond
        // the wall (the node's own, tau_w, less tgx e_x + tgy e_y for the
        // pulled direction), and the rule's result must be relative to the
        // node's own reference (tau_w is the same all along a wall of the
        // reference axis): a Dirichlet wall's constant loses 2 c_i tau_w
        // and gains gdc_i, an adiabatic wall's constant is -gdc_i.
        const int n_side = (s == LBM_LEFT || s == LBM_RIGHT) ? h->nx : h->ny;
        const double tau_w = (s == LBM_LEFT || s == LBM_BOTTOM) ? C.tb : C.tb + (C.tgx + C.tgy) * (n_side - 1);
        for (int i = 0; i < 9; ++i) {
            double c = 0.0;
            if (dir && i > 0) {
                const double Tw = p->wall_T[s];
                if (q9) {
                    const double eu = ex(i) * p->wall_u[s][0] + ey(i) * p->wall_u[s][1];
                    const double usq = p->wall_u[s][0] * p->wall_u[s][0] + p->wall_u[s][1] * p->wall_u[s][1];
                    c = 2.0 * kW9[i] * Tw * (1.0 + p->theta * (4.5 * eu * eu - 1.5 * usq)) - (dev ? 2.0 * kW9[i] * T0 : 0.0);
                } else if (i <= 4) {
                    c = dev ? 0.5 * p->varpi * (Tw - T0) : 0.5 * p->varpi * Tw;
                }
            }
            if (C.tgx != 0.0 || C.tgy != 0.0) {
                if (dir) c += -2.0 * (q9 ? kW9[i] : (i == 0 ? 1.0 - p->varpi : 0.25 * p->varpi)) * tau_w + C.gdc[i];
                else c -= C.gdc[i];
            }
            C.gconst[s][i] = c;
        }
    }
    C.any_nee = nee > 0;
    for (int s = 0; s < 4; ++s) {
        C.nee[s] = p->bc_flow[s] == LBM_BC_NEE;
        C.tdir[s] = p->bc_temp[s] == LBM_T_NEE_DIRICHLET;
        C.uw[s][0] = p->wall_u[s][0];
        C.uw[s][1] = p->wall_u[s][1];
        C.wT[s] = p->wall_T[s];
    }
    C.collision = p->collision;
    fill_rates(C.rd, C);
    fill_rates(C.rf, C);
    C.fscale = C.finv = C.gscale = C.ginv = 1.0f;
    if (h->storage == LBM_F16) {
        // Powers of two: deviations of O(0.1) for fbar and of O(|T - T0|)
        // for g land near 2^9..2^10, far above the FP16 subnormal range and
        // far below its maximum.
        C.fscale = 4096.0f;
        double tr = fabs(p->t_hot - T0);
        for (int s = 0; s < 4; ++s)
            if (p->bc_temp[s] == LBM_T_DIRICHLET || p->bc_temp[s] == LBM_T_NEE_DIRICHLET)
                tr = fmax(tr, fabs(p->wall_T[s] - T0));
        if (!(tr > 0)) tr = 1.0;
        const int k = (int)floor(log2(1024.0 / tr));
        C.gscale = (float)ldexp(1.0, k < -14 ? -14 : (k > 20 ? 20 : k));
        C.finv = 1.0f / C.fscale;
        C.ginv = 1.0f / C.gscale;
    }
    h->G.px = p->bc_flow[LBM_LEFT] == LBM_BC_PERIODIC;
    h->G.py = p->bc_flow[LBM_BOTTOM] == LBM_BC_PERIODIC;
    h->C = C;
    // device copy read by the step kernels, ordered on the solver's stream
    LBM_HIP(h, hipMemcpyAsync(h->d_coeffs, &h->C, sizeof(Coeffs), hipMemcpyHostToDevice, h->stream),
            "copy of the step constants");
    h->s_nu = s_nu;
    h->zeta_alpha = z_a;
    h->gbeta = gbeta;
    h->T0 = T0;
    h->length = length;
    h->dT = dT;
    h->params = *p;
    return LBM_OK;
}

static int reset_rest(lbm_solver* h, const double* T_host) {
    double* dT = nullptr;
    const size_t n = (size_t)h->nx * h->ny;
    if (T_host) {
        LBM_HIP(h, hipMallocAsync(reinterpret_cast<void**>(&dT), n * sizeof(double), h->stream), "hipMallocAsync(T)");
        hipError_t e = hipMemcpyAsync(dT, T_host, n * sizeof(double), hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) {
            (void)hipFreeAsync(dT, h->stream);
            return hip_fail(h, e, "copy of the temperature field");
        }
    }
    hipError_t e = launch_unstream(h->storage, h->ng, h->G, h->C, h->buf[0], nullptr, nullptr, dT, h->T0, true, h->stream);
    if (dT) (void)hipFreeAsync(dT, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "initial-state kernel");
    h->cur = 0;
    h->t = 0;
    h->snap_valid = false;
    if (h->batch) batch_invalidate(h->batch);
    if (T_host) LBM_HIP(h, hipStreamSynchronize(h->stream), "synchronize after initial state");
    return LBM_OK;
}

int lbm_set_params(lbm_solver* h, const lbm_params* p) {
    if (!h) return fail(nullptr, LBM_ERR_ARG, "lbm_set_params: NULL handle");
    if (!p) return fail(h, LBM_ERR_ARG, "lbm_set_params: NULL params");
    if (p->struct_size != sizeof(lbm_params))
        return fail(h, LBM_ERR_ARG, "lbm_set_params: struct_size does not match this library's lbm_params");
    int rc = derive(h, p);
    if (rc != LBM_OK) return rc;
    drop_graphs(h);
    h->params_set = true;
    if (h->batch) batch_invalidate(h->batch);
    return reset_rest(h, nullptr);
}

int lbm_get_derived(const lbm_solver* h, double* s9, double* q9, double* gbeta, double* T0,
                    double* length, double* dT) {
    if (!h) return fail(nullptr, LBM_ERR_ARG, "lbm_get_derived: NULL handle");
    if (!h->params_set) return fail(h, LBM_ERR_STATE, "lbm_get_derived: call lbm_set_params first");
    if (s9) {
        const double s[9] = {1, 1, 1, h->C.s3, h->C.s4, h->C.s4, h->C.s6, h->C.s6, h->C.s8};
        memcpy(s9, s, sizeof(s));
    }
    if (q9) {
        const double C1 = h->C.z1, C3 = h->C.z3, C4 = h->C.z4, C6 = h->C.z6, C8 = h->C.z8;
        const double q5[9] = {1, C1, C1, C3, C4, 0, 0, 0, 0};
        const double q9v[9] = {1, C1, C1, C3, C4, C4, C6, C6, C8};
        const double* q = h->ng == 9 ? q9v : q5;
        for (int k = 0; k < 9; ++k) q9[k] = h->ng == 0 ? 0.0 : q[k];
    }
    if (gbeta) *gbeta = h->gbeta;
    if (T0) *T0 = h->T0;
    if (length) *length = h->length;
    if (dT) *dT = h->dT;
    return LBM_OK;
}

int lbm_init_temperature(lbm_solver* h, const double* T) {
    if (!h) return fail(nullptr, LBM_ERR_ARG, "lbm_init_temperature: NULL handle");
    if (!h->params_set) return fail(h, LBM_ERR_STATE, "lbm_init_temperature: call lbm_set_params first");
    if (T && h->ng == 0)
        return fail(h, LBM_ERR_UNSUPPORTED, "lbm_init_temperature: the isothermal model has no temperature");
    return reset_rest(h, T);
}

// Capture graph_steps sweeps starting from buffer `start` on the solver's
// stream.
// Whether lbm_step may fuse pairs of time steps into one launch: asked for
// by the policy, buffers below 4 GiB, and, with NEE walls, no last tile one
// node wide or high (its wall rebuild would need rows beyond the fused
// tile's halo).
static bool fuse2_active(const lbm_solver* h) {
    if (!h->L.fuse2 || !h->L.buffer) return false;
    if (h->buf_bytes >= (1ull << 32)) return false;
    if (h->C.any_nee) {
        const int ty = fuse2_rows(h->storage, h->ng);
        if (h->nx % 64 == 1 || ty <= 0 || h->ny % ty == 1) return false;
    }
    return true;
}

// Whether lbm_step may run K time steps per launch: asked for by the
// policy, a kernel built for the storage and model, buffers below 4 GiB,
// and, with NEE walls, no last tile one node wide or high.
static bool fusek_active(const lbm_solver* h) {
    if (!h->L.fusek || !h->L.buffer) return false;
    if (h->buf_bytes >= (1ull << 32)) return false;
    const int tx = fusek_tile_cols(h->storage, h->ng), ty = fusek_tile_rows(h->storage, h->ng);
    if (tx <= 0 || ty <= 0) return false;
    if (h->C.any_nee && (h->nx % tx == 1 || h->ny % ty == 1)) return false;
    return true;
}

// Sweeps of `steps` time steps from buffer `cur`; returns the number of
// launches (each swaps the buffers once) or a negative HIP error.
static hipError_t launch_steps(lbm_solver* h, int cur, int64_t steps, int64_t* launches) {
    const bool fuse = fuse2_active(h), fusek = fusek_active(h);
    const int64_t k = fusek_launch_steps(h->storage, h->ng);
    int64_t n = 0;
    while (steps > 0) {
        hipError_t e;
        if (fusek && steps >= k) {
            e = launch_sweepk(h->storage, h->ng, h->L, h->G, h->C, h->d_coeffs, h->buf[cur], h->buf[cur ^ 1],
                              h->stream);
            steps -= k;
        } else if (fuse && steps >= 2) {
            e = launch_sweep2(h->storage, h->ng, h->L, h->G, h->C, h->d_coeffs, h->buf[cur], h->buf[cur ^ 1],
                              h->stream);
            steps -= 2;
        } else {
            e = launch_sweep(h->storage, h->ng, h->L, h->G, h->C, h->d_coeffs, h->buf[cur], h->buf[cur ^ 1],
                             h->stream);
            steps -= 1;
        }
        if (e != hipSuccess) return e;
        cur ^= 1;
        ++n;
    }
    *launches = n;
    return hipSuccess;
}

static int build_graph(lbm_solver* h, int start) {
    hipGraph_t g = nullptr;
    LBM_HIP(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    int64_t launches = 0;
    hipError_t le = launch_steps(h, start, h->graph_steps, &launches);
    h->graph_launches = launches;
    hipError_t ee = hipStreamEndCapture(h->stream, &g);
    if (le != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(h, le, "sweep launch during graph capture");
    }
    if (ee != hipSuccess) return hip_fail(h, ee, "hipStreamEndCapture");
    hipError_t ie = hipGraphInstantiate(&h->graph_exec[start], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
        h->graph_exec[start] = nullptr;
        return hip_fail(h, ie, "hipGraphInstantiate");
    }
    return LBM_OK;
}

// The launches of lbm_step: captured graphs of graph_steps steps while
// enough remain, then single launches; *launched counts kernel launches.
static int step_body(lbm_solver* h, int64_t nsteps, int64_t* launched) {
    if (h->graph_steps > 0) {
        while (nsteps >= h->graph_steps) {
            if (!h->graph_exec[h->cur]) {
                int rc = build_graph(h, h->cur);
                if (rc != LBM_OK) return rc;
            }
            LBM_HIP(h, hipGraphLaunch(h->graph_exec[h->cur], h->stream), "hipGraphLaunch");
            h->t += h->graph_steps;
            h->cur ^= (int)(h->graph_launches & 1);
            nsteps -= h->graph_steps;
            *launched += h->graph_launches;
        }
    }
    if (nsteps > 0) {
        int64_t launches = 0;
        hipError_t e = launch_steps(h, h->cur, nsteps, &launches);
        if (e != hipSuccess) return hip_fail(h, e, "sweep launch");
        h->cur ^= (int)(launches & 1);
        h->t += nsteps;
        *launched += launches;
    }
    return LBM_OK;
}

int lbm_step(lbm_solver* h, int64_t nsteps) {
    if (!h) return fail(nullptr, LBM_ERR_ARG, "lbm_step: NULL handle");
    if (!h->params_set) return fail(h, LBM_ERR_STATE, "lbm_step: call lbm_set_params first");
    if (nsteps < 0) return fail(h, LBM_ERR_ARG, "lbm_step: nsteps < 0");
    if (h->batch && nsteps > 0) batch_invalidate(h->batch);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    const bool prof = h->prof && nsteps > 0 && hipStreamIsCapturing(h->stream, &cap) == hipSuccess &&
                      cap == hipStreamCaptureStatusNone;
    int64_t launched = 0;
    if (!prof) return step_body(h, nsteps, &launched);
    if (h->prof_ev.size() >= 256) prof_drain(h, false);
    if (h->prof_ev.size() >= 256) prof_drain(h, true);
    hipEvent_t ev[2] = {nullptr, nullptr};
    int rc = LBM_OK;
    if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess ||
        hipEventRecord(ev[0], h->stream) != hipSuccess)
        rc = fail(h, LBM_ERR_DEVICE, "lbm_step: profiling events");
    if (rc == LBM_OK) rc = step_body(h, nsteps, &launched);
    if (rc == LBM_OK && hipEventRecord(ev[1], h->stream) != hipSuccess)
        rc = fail(h, LBM_ERR_DEVICE, "lbm_step: profiling events");
    if (rc != LBM_OK) {
        for (hipEvent_t x : ev)
            if (x) (void)hipEventDestroy(x);
        return rc;
    }
    h->prof_ev.push_back(ev[0]);
    h->prof_ev.push_back(ev[1]);
    h->prof_calls += 1;
    h->prof_steps += nsteps;
    h->prof_launches += launched;
    return LBM_OK;
}

int lbm_set_graph_steps(lbm_solver* h, int32_t steps) {
    if (!h) return fail(nullptr, LBM_ERR_ARG, "lbm_set_graph_steps: NULL handle");
    if (steps < 0 || steps % 2 != 0 || steps > 4096)
        return fail(h, LBM_ERR_ARG, "lbm_set_graph_steps: an even count in [0, 4096]");
    drop_graphs(h);
    h->graph_steps = steps;
    return LBM_OK;
}

int lbm_get_graph_steps(const lbm_solver* h, int32_t* steps) {
    if (!h || !steps) return fail(nullptr, LBM_ERR_ARG, "lbm_get_graph_steps: NULL argument");
    *steps = h->graph_steps;
    return LBM_OK;
}

int lbm_time(const lbm_solver* h, int64_t* t) {
    if (!h || !t) return fail(nullptr, LBM_ERR_ARG, "lbm_time: NULL argument");
    *t = h->t;
    return LBM_OK;
}

int lbm_synchronize(lbm_solver* h) {
    if (!h) return fail(nullptr, LBM_ERR_ARG, "lbm_synchronize: NULL handle");
    LBM_HIP(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize");
    return LBM_OK;
}

int lbm_moments_device(lbm_solver* h, double* rho, double* ux, double* uy, double* T) {
    if (!h) return fail(nullptr, LBM_ERR_ARG, "lbm_moments_device: NULL handle");
    if (!h->params_set) return fail(h, LBM_ERR_STATE, "lbm_moments_device: call lbm_set_params first");
    hipError_t e = launch_moments(h->storage, h->ng, h->G, h->C, h->buf[h->cur], rho, ux, uy, T, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "moments kernel");
    return LBM_OK;
}

static int ensure(lbm_solver* h, void** p, size_t bytes, const char* what) {
    if (*p) return LBM_OK;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(h, LBM_ERR_NOMEM, std::string("allocation of ") + what + " failed: " + hipGetErrorString(e));
    }
    return LBM_OK;
}

int lbm_moments(lbm_solver* h, double* rho, double* ux, double* uy, double* T) {
    if (!h) return fail(nullptr, LBM_ERR_ARG, "lbm_moments: NULL handle");
    if (!h->params_set) return fail(h, LBM_ERR_STATE, "lbm_moments: call lbm_set_params first");
    const size_t n = (size_t)h->nx * h->ny;
    int rc = ensure(h, reinterpret_cast<void**>(&h->fields), 4 * n * sizeof(double), "moment staging");
    if (rc != LBM_OK) return rc;
    double* d[4] = {h->fields, h->fields + n, h->fields + 2 * n, h->fields + 3 * n};
    double* o[4] = {rho, ux, uy, T};
    hipError_t e = launch_moments(h->storage, h->ng, h->G, h->C, h->buf[h->cur], rho ? d[0] : nullptr,
                                  ux ? d[1] : nullptr, uy ? d[2] : nullptr, T ? d[3] : nullptr, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "moments kernel");
    for (int k = 0; k < 4; ++k)
        if (o[k]) LBM_HIP(h, hipMemcpyAsync(o[k], d[k], n * sizeof(double), hipMemcpyDeviceToHost, h->stream), "moments copy");
    LBM_HIP(h, hipStreamSynchronize(h->stream), "moments synchronize");
    return LBM_OK;
}

static int nusselt_common(lbm_solver* h, int32_t side, double* host_local, double* out3) {
    if (!h->params_set) return fail(h, LBM_ERR_STATE, "lbm_nusselt: call lbm_set_params first");
    if (side < LBM_LEFT || side > LBM_TOP) return fail(h, LBM_ERR_ARG, "lbm_nusselt: side out of range");
    if (h->ng == 0) return fail(h, LBM_ERR_UNSUPPORTED, "lbm_nusselt: the isothermal model has no temperature");
    const int nee = h->params.bc_temp[side] == LBM_T_NEE_DIRICHLET;
    if (h->params.bc_temp[side] != LBM_T_DIRICHLET && !nee)
        return fail(h, LBM_ERR_ARG, "lbm_nusselt: the side is not a Dirichlet wall");
    const int depth = (side == LBM_LEFT || side == LBM_RIGHT) ? h->nx : h->ny;
    const int count = (side == LBM_LEFT || side == LBM_RIGHT) ? h->ny : h->nx;
    if (depth < 2 + nee) return fail(h, LBM_ERR_ARG, "lbm_nusselt: the lattice is too shallow at this wall");
    if (!(h->dT != 0)) return fail(h, LBM_ERR_ARG, "lbm_nusselt: t_hot == t_cold");
    int rc = ensure(h, reinterpret_cast<void**>(&h->nu_local),
                    (size_t)(h->nx > h->ny ? h->nx : h->ny) * sizeof(double), "Nusselt staging");
    if (rc != LBM_OK) return rc;
    hipError_t e = launch_nusselt(h->storage, h->ng, h->G, h->C, h->buf[h->cur], side, h->params.wall_T[side],
                                  h->length, h->dT, nee, h->nu_local, h->small, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "Nusselt kernel");
    LBM_HIP(h, hipMemcpyAsync(h->host_small, h->small, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream), "Nusselt copy");
    if (host_local)
        LBM_HIP(h, hipMemcpyAsync(host_local, h->nu_local, (size_t)count * sizeof(double), hipMemcpyDeviceToHost, h->stream), "Nusselt copy");
    LBM_HIP(h, hipStreamSynchronize(h->stream), "Nusselt synchronize");
    memcpy(out3, h->host_small, 3 * sizeof(double));
    return LBM_OK;
}

int lbm_nusselt(lbm_solver* h, int32_t side, double* nu_mean, double* nu_max, int32_t* i_max) {
    if (!h) return fail(nullptr, LBM_ERR_ARG, "lbm_nusselt: NULL handle");
    double o[3];
    int rc = nusselt_common(h, side, nullptr, o);
    if (rc != LBM_OK) return rc;
    if (nu_mean) *nu_mean = o[0];
    if (nu_max) *nu_max = o[1];
    if (i_max) *i_max = (int32_t)o[2];
    return LBM_OK;
}

int lbm_nusselt_local(lbm_solver* h, int32_t side, double* nu_local) {
    if (!h) return fail(nullptr, LBM_ERR_ARG, "lbm_nusselt_local: NULL handle");
    if (!nu_local) return fail(h, LBM_ERR_ARG, "lbm_nusselt_local: NULL output");
    double o[3];
    return nusselt_common(h, side, nu_local, o);
}

// The residual kernels on the handle's snapshot with the given partials
// and reduced outputs (2 doubles, device), then the host readout.
static int residual_run(lbm_solver* h, double* pmax, unsigned long long* pbad, double* out2, const char* who,
                        double* r, int64_t* nonfinite) {
    const bool first = !h->snap_valid;
    hipError_t e = launch_residual(h->storage, h->ng, h->G, h->C, h->buf[h->cur], h->snap, first, pmax, pbad, out2,
                                   h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "residual kernels");
    LBM_HIP(h, hipMemcpyAsync(h->host_small + 4, out2, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream), "residual copy");
    LBM_HIP(h, hipStreamSynchronize(h->stream), "residual synchronize");
    h->snap_valid = true;
    const double rv = first ? INFINITY : h->host_small[4];
    const int64_t bad = (int64_t)h->host_small[5];
    if (r) *r = rv;
    if (nonfinite) *nonfinite = bad;
    if (bad) return fail(h, LBM_ERR_UNSTABLE, std::string(who) + ": non-finite values in the lattice");
    return LBM_OK;
}

int lbm_residual(lbm_solver* h, double* r, int64_t* nonfinite) {
    if (!h) return fail(nullptr, LBM_ERR_ARG, "lbm_residual: NULL handle");
    if (!h->params_set) return fail(h, LBM_ERR_STATE, "lbm_residual: call lbm_set_params first");
    const size_t n = (size_t)h->nx * h->ny;
    int rc = ensure(h, reinterpret_cast<void**>(&h->snap), 3 * n * sizeof(double), "residual snapshot");
    if (rc == LBM_OK) rc = ensure(h, reinterpret_cast<void**>(&h->rpart), residual_parts(h->G) * sizeof(double), "residual partials");
    if (rc == LBM_OK) rc = ensure(h, reinterpret_cast<void**>(&h->rbad), residual_parts(h->G) * sizeof(unsigned long long), "residual partials");
    if (rc != LBM_OK) return rc;
    return residual_run(h, h->rpart, h->rbad, h->small + 4, "lbm_residual", r, nonfinite);
}

// ---------------------------------------------------------------------------
// The residual without allocation (lbm_residual_static).  Its per-block
// partial maxima and non-finite counts and the two reduced values live in
// `scratch`, a static device array that each GPU the library runs on holds
// until the process ends, instead of buffers the handle allocates on first
// use.  Host code never passes `scratch` itself (on the host the name is
// only a stand-in for the device symbol): the device address of each GPU's
// copy is looked up once, with that GPU current, and kept per device.
// Every call on one GPU shares that GPU's copy; calls that overlap on one
// GPU (other threads, or other streams before a call has synchronized)
// race on it.  Nothing in it needs clearing: each partial is written by its
// block before the final reduction reads it.
// ---------------------------------------------------------------------------
namespace {
constexpr int kStaticParts = 65536;   // one partial per 256 nodes: lattices up to 2^24 nodes
constexpr size_t kStaticOut = (size_t)kStaticParts * (sizeof(double) + sizeof(unsigned long long));
constexpr size_t kScratchBytes = kStaticOut + 256;   // partials, then the two reduced values
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static hipError_t scratch_on(int dev, char** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int prev = -1;
        hipError_t e = hipGetDevice(&prev);
        if (e == hipSuccess && prev != dev) e = hipSetDevice(dev);
        void* p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<char*>(g_scratch_ptr[dev]);
    return hipSuccess;
}

int lbm_residual_static(lbm_solver* h, double* r, int64_t* nonfinite) {
    if (!h) return fail(nullptr, LBM_ERR_ARG, "lbm_residual_static: NULL handle");
    if (!h->params_set) return fail(h, LBM_ERR_STATE, "lbm_residual_static: call lbm_set_params first");
    if (!h->snap)
        return fail(h, LBM_ERR_STATE, "lbm_residual_static: the handle has no residual snapshot yet "
                                      "(lbm_residual or lbm_batch_add allocates it)");
    const int nb = residual_parts(h->G);
    if (nb > kStaticParts)
        return fail(h, LBM_ERR_ARG, "lbm_residual_static: " + std::to_string((long long)h->nx * h->ny) +
                                        " nodes; the static scratch serves lattices of at most 16777216 nodes");
    if (h->device < 0 || h->device >= kMaxDevices)
        return fail(h, LBM_ERR_DEVICE, "lbm_residual_static: device id outside 0..63");
    char* base = nullptr;
    hipError_t e = scratch_on(h->device, &base);
    if (e != hipSuccess) return hip_fail(h, e, "lbm_residual_static: address of the static scratch");
    return residual_run(h, reinterpret_cast<double*>(base),
                        reinterpret_cast<unsigned long long*>(base + (size_t)kStaticParts * sizeof(double)),
                        reinterpret_cast<double*>(base + kStaticOut), "lbm_residual_static", r, nonfinite);
}

int lbm_get_populations(lbm_solver* h, double* f9, double* g5) {
    if (!h) return fail(nullptr, LBM_ERR_ARG, "lbm_get_populations: NULL handle");
    if (!h->params_set) return fail(h, LBM_ERR_STATE, "lbm_get_populations: call lbm_set_params first");
    const size_t n = (size_t)h->nx * h->ny;
    double* d = nullptr;
    LBM_HIP(h, hipMallocAsync(reinterpret_cast<void**>(&d), (9 + h->ng) * n * sizeof(double), h->stream), "hipMallocAsync(populations)");
    hipError_t e = launch_gather(h->storage, h->ng, h->G, h->C, h->buf[h->cur], d, d + 9 * n, h->T0, h->stream);
    if (e == hipSuccess && f9) e = hipMemcpyAsync(f9, d, 9 * n * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && g5 && h->ng)
        e = hipMemcpyAsync(g5, d + 9 * n, h->ng * n * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    (void)hipFreeAsync(d, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "lbm_get_populations");
    LBM_HIP(h, hipStreamSynchronize(h->stream), "populations synchronize");
    return LBM_OK;
}

int lbm_set_populations(lbm_solver* h, const double* f9, const double* g5) {
    if (!h) return fail(nullptr, LBM_ERR_ARG, "lbm_set_populations: NULL handle");
    if (!f9 || (!g5 && h->ng)) return fail(h, LBM_ERR_ARG, "lbm_set_populations: NULL input");
    if (!h->params_set) return fail(h, LBM_ERR_STATE, "lbm_set_populations: call lbm_set_params first");
    const size_t n = (size_t)h->nx * h->ny;
    double* d = nullptr;
    LBM_HIP(h, hipMallocAsync(reinterpret_cast<void**>(&d), (9 + h->ng) * n * sizeof(double), h->stream), "hipMallocAsync(populations)");
    hipError_t e = hipMemcpyAsync(d, f9, 9 * n * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && h->ng)
        e = hipMemcpyAsync(d + 9 * n, g5, h->ng * n * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = launch_unstream(h->storage, h->ng, h->G, h->C, h->buf[h->cur], d, d + 9 * n, nullptr, h->T0, false, h->stream);
    (void)hipFreeAsync(d, h->stream);
    if (e != hipSuccess) return hip_fail(h, e, "lbm_set_populations");
    LBM_HIP(h, hipStreamSynchronize(h->stream), "populations synchronize");
    h->snap_valid = false;
    return LBM_OK;
}

// Saved state: a header, then the current population buffer.
struct StateHeader {
    uint64_t magic;
    int32_t nx, ny, storage, pitch;
    int64_t plane, t;
    uint64_t buf_bytes;
};
static const uint64_t kStateMagic = 0x4c424d5354415431ull;  // "LBMSTAT1"

int lbm_state_bytes(const lbm_solver* h, uint64_t* bytes) {
    if (!h || !bytes) return fail(nullptr, LBM_ERR_ARG, "lbm_state_bytes: NULL argument");
    *bytes = sizeof(StateHeader) + h->buf_bytes;
    return LBM_OK;
}

int lbm_save_state(lbm_solver* h, void* host, uint64_t bytes) {
    if (!h) return fail(nullptr, LBM_ERR_ARG, "lbm_save_state: NULL handle");
    if (!host || bytes < sizeof(StateHeader) + h->buf_bytes) return fail(h, LBM_ERR_ARG, "lbm_save_state: buffer too small");
    if (!h->params_set) return fail(h, LBM_ERR_STATE, "lbm_save_state: call lbm_set_params first");
    StateHeader hd{kStateMagic, h->nx, h->ny, h->storage, h->G.pitch, h->G.plane, h->t, h->buf_bytes};
    memcpy(host, &hd, sizeof(hd));
    LBM_HIP(h, hipMemcpyAsync(static_cast<char*>(host) + sizeof(hd), h->buf[h->cur], h->buf_bytes, hipMemcpyDeviceToHost, h->stream), "state copy");
    LBM_HIP(h, hipStreamSynchronize(h->stream), "state synchronize");
    return LBM_OK;
}

int lbm_load_state(lbm_solver* h, const void* host, uint64_t bytes) {
    if (!h) return fail(nullptr, LBM_ERR_ARG, "lbm_load_state: NULL handle");
    if (!h->params_set) return fail(h, LBM_ERR_STATE, "lbm_load_state: call lbm_set_params first");
    if (!host || bytes < sizeof(StateHeader)) return fail(h, LBM_ERR_ARG, "lbm_load_state: buffer too small");
    StateHeader hd;
    memcpy(&hd, host, sizeof(hd));
    if (hd.magic != kStateMagic || hd.nx != h->nx || hd.ny != h->ny || hd.storage != h->storage ||
        hd.pitch != h->G.pitch || hd.plane != h->G.plane || hd.buf_bytes != h->buf_bytes ||
        bytes < sizeof(hd) + h->buf_bytes)
        return fail(h, LBM_ERR_ARG, "lbm_load_state: the state was saved from a different lattice or storage");
    LBM_HIP(h, hipMemcpyAsync(h->buf[h->cur], static_cast<const char*>(host) + sizeof(hd), h->buf_bytes, hipMemcpyHostToDevice, h->stream), "state copy");
    LBM_HIP(h, hipStreamSynchronize(h->stream), "state synchronize");
    if (h->batch) batch_invalidate(h->batch);
    h->t = hd.t;
    h->snap_valid = false;
    return LBM_OK;
}

int lbm_set_launch(lbm_solver* h, int32_t block_x, int32_t block_y, int32_t rows_per_thread, int32_t policy) {
    if (!h) return fail(nullptr, LBM_ERR_ARG, "lbm_set_launch: NULL handle");
    Launch L = h->L;
    if (block_x) L.bx = block_x;
    if (block_y) L.by = block_y;
    if (rows_per_thread) L.rows = rows_per_thread;
    if (!(L.bx == 64 || L.bx == 128 || L.bx == 256) || L.by < 1 || L.bx * L.by > 256 ||
        !(L.rows == 1 || L.rows == 2))
        return fail(h, LBM_ERR_ARG, "lbm_set_launch: block_x in {64,128,256}, block_x*block_y <= 256, rows in {1,2}");
    if (policy < LBM_POLICY_DEFAULT ||
        policy > (LBM_POLICY_XCD_BANDS | LBM_POLICY_KEEP_STORES | LBM_POLICY_XCD_STRIPS | LBM_POLICY_FUSE2 |
                  LBM_POLICY_FUSEK) ||
        (policy >= 0 && (policy & LBM_POLICY_XCD_BANDS) && (policy & LBM_POLICY_XCD_STRIPS)))
        return fail(h, LBM_ERR_ARG, "lbm_set_launch: unknown policy (bands and strips exclude each other)");
    h->L = L;
    if (policy == LBM_POLICY_DEFAULT) {
        default_policy(h);
    } else if (policy >= 0) {
        h->L.order = (policy & LBM_POLICY_XCD_BANDS) ? 1 : ((policy & LBM_POLICY_XCD_STRIPS) ? 2 : 0);
        h->L.keep = (policy & LBM_POLICY_KEEP_STORES) != 0;
        h->L.fuse2 = (policy & LBM_POLICY_FUSE2) != 0;
        h->L.fusek = (policy & LBM_POLICY_FUSEK) != 0;
    }
    drop_graphs(h);
    if (h->batch) batch_invalidate(h->batch);
    return LBM_OK;
}

int lbm_steps_per_launch(const lbm_solver* h, int32_t* steps) {
    if (!h || !steps) return fail(nullptr, LBM_ERR_ARG, "lbm_steps_per_launch: NULL argument");
    *steps = fusek_active(h) ? fusek_launch_steps(h->storage, h->ng) : (fuse2_active(h) ? 2 : 1);
    return LBM_OK;
}

int lbm_get_launch(const lbm_solver* h, int32_t* block_x, int32_t* block_y, int32_t* rows_per_thread,
                   int32_t* policy) {
    if (!h) return fail(nullptr, LBM_ERR_ARG, "lbm_get_launch: NULL handle");
    if (block_x) *block_x = h->L.bx;
    if (block_y) *block_y = h->L.by;
    if (rows_per_thread) *rows_per_thread = h->L.rows;
    if (policy)
        *policy = (h->L.order == 1 ? LBM_POLICY_XCD_BANDS : 0) | (h->L.order == 2 ? LBM_POLICY_XCD_STRIPS : 0) |
                  (h->L.keep ? LBM_POLICY_KEEP_STORES : 0) | (h->L.fuse2 ? LBM_POLICY_FUSE2 : 0) |
                  (h->L.fusek ? LBM_POLICY_FUSEK : 0);
    return LBM_OK;
}


// ---------------------------------------------------------------------------
// Batches: many independent lattices advanced by one launch per step.
// ---------------------------------------------------------------------------
static int bfail(lbm_batch* b, int code, const std::string& msg) {
    if (b) b->err = msg;
    else g_create_error = msg;
    return code;
}

static void batch_drop_graphs(lbm_batch* b) {
    for (int k = 0; k < 2; ++k) {
        if (b->graph_exec[k]) (void)hipGraphExecDestroy(b->graph_exec[k]);
        b->graph_exec[k] = nullptr;
    }
}

static void batch_invalidate(lbm_batch* b) {
    b->dirty = true;
    batch_drop_graphs(b);
}

int lbm_batch_create(lbm_batch** out, int32_t storage, void* hip_stream) {
    if (!out) return bfail(nullptr, LBM_ERR_ARG, "lbm_batch_create: NULL output handle");
    *out = nullptr;
    if (storage < LBM_F64 || storage > LBM_F16) return bfail(nullptr, LBM_ERR_ARG, "lbm_batch_create: bad storage");
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return bfail(nullptr, LBM_ERR_NOMEM, "lbm_batch_create: host allocation failed");
    b->storage = storage;
    if (hip_stream) {
        b->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete b;
            return bfail(nullptr, LBM_ERR_DEVICE, std::string("lbm_batch_create: stream: ") + hipGetErrorString(e));
        }
        b->own_stream = true;
    }
    *out = b;
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (auto* m : b->slots)
        if (m) m->batch = nullptr;
    batch_drop_graphs(b);
    if (b->d_members) (void)hipFree(b->d_members);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_ftiles) (void)hipFree(b->d_ftiles);
    if (b->d_fktiles) (void)hipFree(b->d_fktiles);
    if (b->d_tile_max) (void)hipFree(b->d_tile_max);
    if (b->d_tile_bad) (void)hipFree(b->d_tile_bad);
    if (b->d_rout) (void)hipFree(b->d_rout);
    if (b->h_rout) (void)hipHostFree(b->h_rout);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err.c_str() : g_create_error.c_str(); }
void* lbm_batch_stream(const lbm_batch* b) { return b ? static_cast<void*>(b->stream) : nullptr; }

int lbm_batch_add(lbm_batch* b, lbm_solver* h, int32_t* slot) {
    if (!b || !h) return bfail(b, LBM_ERR_ARG, "lbm_batch_add: NULL argument");
    if (h->batch) return bfail(b, LBM_ERR_STATE, "lbm_batch_add: the solver already belongs to a batch");
    if (h->storage != b->storage) return bfail(b, LBM_ERR_ARG, "lbm_batch_add: storage differs from the batch's");
    int active = 0;
    for (auto* m : b->slots) active += m != nullptr;
    if (active && h->ng != b->ng) return bfail(b, LBM_ERR_ARG, "lbm_batch_add: thermal model differs from the batch's");
    if (h->stream != b->stream) return bfail(b, LBM_ERR_ARG, "lbm_batch_add: the solver must use the batch's stream");
    if (!h->params_set) return bfail(b, LBM_ERR_STATE, "lbm_batch_add: call lbm_set_params on the solver first");
    if (h->C.collision != LBM_COLLISION_MRT)
        return bfail(b, LBM_ERR_UNSUPPORTED, "lbm_batch_add: batch members use the MRT collision");
    // members keep a residual snapshot so that the batch can take every
    // member's residual in one launch
    if (ensure(h, reinterpret_cast<void**>(&h->snap), 3 * (size_t)h->nx * h->ny * sizeof(double),
               "residual snapshot") != LBM_OK)
        return bfail(b, LBM_ERR_NOMEM, h->err);
    int k = 0;
    while (k < (int)b->slots.size() && b->slots[k]) ++k;
    if (k == (int)b->slots.size()) b->slots.push_back(nullptr);
    b->slots[k] = h;
    h->batch = b;
    b->ng = h->ng;
    batch_invalidate(b);
    if (slot) *slot = k;
    return LBM_OK;
}

int lbm_batch_remove(lbm_batch* b, int32_t slot) {
    if (!b) return bfail(nullptr, LBM_ERR_ARG, "lbm_batch_remove: NULL batch");
    if (slot < 0 || slot >= (int)b->slots.size() || !b->slots[slot])
        return bfail(b, LBM_ERR_ARG, "lbm_batch_remove: empty or invalid slot");
    // work queued for this member must finish before the caller may free it
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, LBM_ERR_DEVICE, std::string("lbm_batch_remove: synchronize: ") + hipGetErrorString(e));
    b->slots[slot]->batch = nullptr;
    b->slots[slot] = nullptr;
    batch_invalidate(b);
    return LBM_OK;
}

int lbm_batch_size(const lbm_batch* b, int32_t* active, int32_t* slots) {
    if (!b) return bfail(nullptr, LBM_ERR_ARG, "lbm_batch_size: NULL batch");
    int a = 0;
    for (auto* m : b->slots) a += m != nullptr;
    if (active) *active = a;
    if (slots) *slots = (int32_t)b->slots.size();
    return LBM_OK;
}

lbm_solver* lbm_batch_member(const lbm_batch* b, int32_t slot) {
    if (!b || slot < 0 || slot >= (int)b->slots.size()) return nullptr;
    return b->slots[slot];
}

// Reallocates a device table to hold n entries if it is too small.
extern "C++" template <class T>
static hipError_t batch_table(T** d, size_t* cap, size_t n) {
    if (n <= *cap) return hipSuccess;
    if (*d) (void)hipFree(*d);
    *d = nullptr;
    *cap = 0;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(d), n * sizeof(T));
    if (e == hipSuccess) *cap = n;
    return e;
}

static int batch_build(lbm_batch* b) {
    std::vector<BatchMember> mem;
    std::vector<BatchTile> tiles, ftiles, fktiles;
    b->member_slot.clear();
    b->buffer = true;
    const int fty = fuse2_rows(b->storage, b->ng < 0 ? 5 : b->ng);
    const int ng = b->ng < 0 ? 5 : b->ng;
    const int ktx = fusek_tile_cols(b->storage, ng), kty = fusek_tile_rows(b->storage, ng);
    bool can_fuse = fty > 0, can_fusek = ktx > 0 && kty > 0;
    double ws = 0.0;
    // members in table order: as added, or the largest lattices first (their
    // tiles then start the launch and the small ones fill its tail)
    std::vector<size_t> order;
    for (size_t k = 0; k < b->slots.size(); ++k)
        if (b->slots[k]) order.push_back(k);
    if (b->tune_sort == 1)
        std::stable_sort(order.begin(), order.end(), [b](size_t a, size_t c) {
            return (long long)b->slots[a]->nx * b->slots[a]->ny > (long long)b->slots[c]->nx * b->slots[c]->ny;
        });
    for (size_t k : order) {
        lbm_solver* h = b->slots[k];
        BatchMember M{};
        M.G = h->G;
        M.C = h->C;
        M.buf[0] = h->buf[0];
        M.buf[1] = h->buf[1];
        M.buf_bytes = h->buf_bytes < (1ull << 32) ? (unsigned)h->buf_bytes : 0u;
        if (h->buf_bytes >= (1ull << 32)) b->buffer = false;
        M.cur0 = h->cur;
        M.snap = h->snap;
        const int id = (int)mem.size();
        M.tile0 = (int)tiles.size();
        const int bx = h->L.bx, by = 256 / h->L.bx;
        for (int y0 = 0; y0 < h->ny; y0 += by)
            for (int x0 = 0; x0 < h->nx; x0 += bx) tiles.push_back(BatchTile{id, x0, y0, bx});
        M.ntiles = (int)tiles.size() - M.tile0;
        for (int y0 = 0; y0 < h->ny; y0 += fty)
            for (int x0 = 0; x0 < h->nx; x0 += 64) ftiles.push_back(BatchTile{id, x0, y0, 64});
        if (can_fusek)
            for (int y0 = 0; y0 < h->ny; y0 += kty)
                for (int x0 = 0; x0 < h->nx; x0 += ktx) fktiles.push_back(BatchTile{id, x0, y0, ktx});
        // a wall node rebuilt by extrapolation must find its fluid
        // neighbour inside the same fused tile
        if (h->C.any_nee && (h->nx % 64 == 1 || h->ny % fty == 1)) can_fuse = false;
        if (h->C.any_nee && can_fusek && (h->nx % ktx == 1 || h->ny % kty == 1)) can_fusek = false;
        ws += 2.0 * (double)h->buf_bytes;
        mem.push_back(M);
        b->member_slot.push_back((int)k);
    }
    // Fused pairs win for FP64 and FP32 batches at every member size
    // measured on MI355X (batches of equal square cavities, 6.7e6 nodes in
    // all, sides 64 to 1024: FP32 1.1x to 1.6x, FP64 1.3x to 1.9x over one
    // step per launch); FP16 batches keep single steps, like FP16 lattices.
    const double mib = 1024.0 * 1024.0;
    // K steps per launch for FP64 batches (batches of equal cavities,
    // 6.7e6 nodes in all: 9-31% less time per step than fused pairs, sides
    // 64 to 1024; the D2Q9 thermal model 7-19% less at sides 64, 256, 512
    // and 1024, 5% more at 128; single FP64 lattices gain at every size);
    // FP32 batches keep fused pairs, which were up to 16% faster at sides
    // 128 to 512 (the margins of small members take the general path; K
    // steps won by 3-14% at sides 64, 96 and 1024).
    const bool want = b->policy == LBM_POLICY_DEFAULT
                          ? (b->storage == LBM_F64 || b->storage == LBM_F32)
                          : (b->policy & LBM_POLICY_FUSE2) != 0;
    const bool wantk = b->policy == LBM_POLICY_DEFAULT ? b->storage == LBM_F64 : (b->policy & LBM_POLICY_FUSEK) != 0;
    b->fuse = want && can_fuse && b->buffer && !mem.empty();
    b->fusek = wantk && can_fusek && b->buffer && !mem.empty();
    b->keep = b->tune_keep < 0 ? ws <= 256.0 * mib : b->tune_keep == 1;
    b->order = b->tune_order < 0 ? 1 : b->tune_order;
    if (batch_table(&b->d_members, &b->cap_members, mem.size()) != hipSuccess)
        return bfail(b, LBM_ERR_NOMEM, "batch member table allocation");
    if (batch_table(&b->d_tiles, &b->cap_tiles, tiles.size()) != hipSuccess)
        return bfail(b, LBM_ERR_NOMEM, "batch tile table allocation");
    if (b->fuse && batch_table(&b->d_ftiles, &b->cap_ftiles, ftiles.size()) != hipSuccess)
        return bfail(b, LBM_ERR_NOMEM, "batch fused tile table allocation");
    if (b->fusek && batch_table(&b->d_fktiles, &b->cap_fktiles, fktiles.size()) != hipSuccess)
        return bfail(b, LBM_ERR_NOMEM, "batch multi-step tile table allocation");
    if (!mem.empty()) {
        hipError_t e = hipMemcpyAsync(b->d_members, mem.data(), mem.size() * sizeof(BatchMember), hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->d_tiles, tiles.data(), tiles.size() * sizeof(BatchTile), hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess && b->fuse)
            e = hipMemcpyAsync(b->d_ftiles, ftiles.data(), ftiles.size() * sizeof(BatchTile), hipMemcpyHostToDevice,
                               b->stream);
        if (e == hipSuccess && b->fusek)
            e = hipMemcpyAsync(b->d_fktiles, fktiles.data(), fktiles.size() * sizeof(BatchTile),
                               hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);   // host vectors die on return
        if (e != hipSuccess) return bfail(b, LBM_ERR_DEVICE, std::string("batch table upload: ") + hipGetErrorString(e));
    }
    b->ntiles = (int)tiles.size();
    b->nftiles = b->fuse ? (int)ftiles.size() : 0;
    b->nfktiles = b->fusek ? (int)fktiles.size() : 0;
    b->parity = 0;
    b->dirty = false;
    return LBM_OK;
}

// Launches for `steps` time steps starting at tile-table parity `parity`
// (fused pairs while two or more steps remain); each launch swaps every
// member's buffers once.  Returns the number of launches in *launches.
static hipError_t batch_launch_steps(lbm_batch* b, int parity, int64_t steps, int64_t* launches) {
    int64_t n = 0;
    const int64_t k = fusek_launch_steps(b->storage, b->ng < 0 ? 5 : b->ng);
    while (steps > 0) {
        hipError_t e;
        if (b->fusek && steps >= k) {
            e = launch_sweepk_batch(b->storage, b->ng, b->keep, b->d_members, b->d_fktiles, b->nfktiles, parity,
                                    b->order, b->stream);
            steps -= k;
        } else if (b->fuse && steps >= 2) {
            e = launch_sweep2_batch(b->storage, b->ng, b->keep, b->d_members, b->d_ftiles, b->nftiles, parity, b->order,
                                    b->stream);
            steps -= 2;
        } else {
            e = launch_sweep_batch(b->storage, b->ng, b->buffer, b->keep, b->d_members, b->d_tiles, b->ntiles, parity,
                                   b->order, b->stream);
            steps -= 1;
        }
        if (e != hipSuccess) return e;
        parity ^= 1;
        ++n;
    }
    *launches = n;
    return hipSuccess;
}

static int batch_build_graph(lbm_batch* b, int start) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bfail(b, LBM_ERR_DEVICE, "batch graph capture begin");
    int64_t launches = 0;
    hipError_t le = batch_launch_steps(b, start, b->graph_steps, &launches);
    b->graph_launches = launches;
    e = hipStreamEndCapture(b->stream, &g);
    if (le != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return bfail(b, LBM_ERR_DEVICE, "batch graph capture");
    }
    e = hipGraphInstantiate(&b->graph_exec[start], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->graph_exec[start] = nullptr;
        return bfail(b, LBM_ERR_DEVICE, "batch graph instantiate");
    }
    return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int64_t nsteps) {
    if (!b) return bfail(nullptr, LBM_ERR_ARG, "lbm_batch_step: NULL batch");
    if (nsteps < 0) return bfail(b, LBM_ERR_ARG, "lbm_batch_step: nsteps < 0");
    if (b->dirty) {
        int rc = batch_build(b);
        if (rc != LBM_OK) return rc;
    }
    int64_t left = nsteps, launches = 0;
    if (b->graph_steps > 0 && b->ntiles > 0) {
        while (left >= b->graph_steps) {
            if (!b->graph_exec[b->parity]) {
                int rc = batch_build_graph(b, b->parity);
                if (rc != LBM_OK) return rc;
            }
            hipError_t e = hipGraphLaunch(b->graph_exec[b->parity], b->stream);
            if (e != hipSuccess) return bfail(b, LBM_ERR_DEVICE, "batch graph launch");
            left -= b->graph_steps;
            launches += b->graph_launches;
            b->parity ^= (int)(b->graph_launches & 1);
        }
    }
    int64_t n = 0;
    hipError_t e = batch_launch_steps(b, b->parity, left, &n);
    if (e != hipSuccess) return bfail(b, LBM_ERR_DEVICE, std::string("batched sweep launch: ") + hipGetErrorString(e));
    b->parity ^= (int)(n & 1);
    launches += n;
    for (auto* h : b->slots) {
        if (!h) continue;
        h->t += nsteps;
        h->cur ^= (int)(launches & 1);
    }
    return LBM_OK;
}

int lbm_batch_set_policy(lbm_batch* b, int32_t policy) {
    if (!b) return bfail(nullptr, LBM_ERR_ARG, "lbm_batch_set_policy: NULL batch");
    if (policy != LBM_POLICY_DEFAULT && (policy < 0 || (policy & ~(LBM_POLICY_FUSE2 | LBM_POLICY_FUSEK)) != 0))
        return bfail(b, LBM_ERR_ARG,
                     "lbm_batch_set_policy: LBM_POLICY_DEFAULT or a mask of LBM_POLICY_FUSE2 and LBM_POLICY_FUSEK");
    b->policy = policy;
    batch_invalidate(b);
    return LBM_OK;
}

int lbm_batch_set_tuning(lbm_batch* b, int32_t xcd_order, int32_t keep_stores, int32_t largest_first) {
    if (!b) return bfail(nullptr, LBM_ERR_ARG, "lbm_batch_set_tuning: NULL batch");
    if (xcd_order < -1 || xcd_order > 1 || keep_stores < -1 || keep_stores > 1 || largest_first < 0 ||
        largest_first > 1)
        return bfail(b, LBM_ERR_ARG, "lbm_batch_set_tuning: xcd_order and keep_stores in -1..1, largest_first 0 or 1");
    b->tune_order = xcd_order;
    b->tune_keep = keep_stores;
    b->tune_sort = largest_first;
    batch_invalidate(b);
    return LBM_OK;
}

int lbm_batch_get_tuning(lbm_batch* b, int32_t* xcd_order, int32_t* keep_stores, int32_t* largest_first) {
    if (!b || !xcd_order || !keep_stores || !largest_first)
        return bfail(b, LBM_ERR_ARG, "lbm_batch_get_tuning: NULL argument");
    if (b->dirty) {
        int rc = batch_build(b);
        if (rc != LBM_OK) return rc;
    }
    *xcd_order = b->order;
    *keep_stores = b->keep ? 1 : 0;
    *largest_first = b->tune_sort;
    return LBM_OK;
}

int lbm_batch_steps_per_launch(lbm_batch* b, int32_t* steps) {
    if (!b || !steps) return bfail(b, LBM_ERR_ARG, "lbm_batch_steps_per_launch: NULL argument");
    if (b->dirty) {
        int rc = batch_build(b);
        if (rc != LBM_OK) return rc;
    }
    *steps = b->fusek ? fusek_launch_steps(b->storage, b->ng < 0 ? 5 : b->ng) : (b->fuse ? 2 : 1);
    return LBM_OK;
}

int lbm_batch_set_graph_steps(lbm_batch* b, int32_t steps) {
    if (!b) return bfail(nullptr, LBM_ERR_ARG, "lbm_batch_set_graph_steps: NULL batch");
    if (steps < 0 || steps % 2 != 0 || steps > 4096)
        return bfail(b, LBM_ERR_ARG, "lbm_batch_set_graph_steps: an even count in [0, 4096]");
    batch_drop_graphs(b);
    b->graph_steps = steps;
    return LBM_OK;
}

int lbm_batch_synchronize(lbm_batch* b) {
    if (!b) return bfail(nullptr, LBM_ERR_ARG, "lbm_batch_synchronize: NULL batch");
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, LBM_ERR_DEVICE, std::string("batch synchronize: ") + hipGetErrorString(e));
    return LBM_OK;
}

int lbm_batch_residual(lbm_batch* b, double* r, int64_t* nonfinite) {
    if (!b) return bfail(nullptr, LBM_ERR_ARG, "lbm_batch_residual: NULL batch");
    if (b->dirty) {
        int rc = batch_build(b);
        if (rc != LBM_OK) return rc;
    }
    const size_t nm = b->member_slot.size();
    if (b->cap_rtiles < (size_t)b->ntiles) {
        if (b->d_tile_max) (void)hipFree(b->d_tile_max);
        if (b->d_tile_bad) (void)hipFree(b->d_tile_bad);
        b->d_tile_max = nullptr;
        b->d_tile_bad = nullptr;
        b->cap_rtiles = 0;
        if (hipMalloc(reinterpret_cast<void**>(&b->d_tile_max), b->ntiles * sizeof(double)) != hipSuccess ||
            hipMalloc(reinterpret_cast<void**>(&b->d_tile_bad), b->ntiles * sizeof(unsigned long long)) != hipSuccess)
            return bfail(b, LBM_ERR_NOMEM, "batch residual scratch");
        b->cap_rtiles = b->ntiles;
    }
    if (b->cap_rout < nm) {
        if (b->d_rout) (void)hipFree(b->d_rout);
        if (b->h_rout) (void)hipHostFree(b->h_rout);
        b->d_rout = nullptr;
        b->h_rout = nullptr;
        b->cap_rout = 0;
        if (hipMalloc(reinterpret_cast<void**>(&b->d_rout), 2 * nm * sizeof(double)) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&b->h_rout), 2 * nm * sizeof(double), hipHostMallocDefault) != hipSuccess)
            return bfail(b, LBM_ERR_NOMEM, "batch residual output");
        b->cap_rout = nm;
    }
    if (nm) {
        hipError_t e = launch_residual_batch(b->storage, b->ng, b->d_members, (int)nm, b->d_tiles, b->ntiles, b->parity,
                                             b->d_tile_max, b->d_tile_bad, b->d_rout, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->h_rout, b->d_rout, 2 * nm * sizeof(double), hipMemcpyDeviceToHost, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return bfail(b, LBM_ERR_DEVICE, std::string("batch residual: ") + hipGetErrorString(e));
    }
    for (size_t k = 0; k < b->slots.size(); ++k) {
        if (r) r[k] = NAN;
        if (nonfinite) nonfinite[k] = -1;
    }
    int worst = LBM_OK;
    for (size_t m = 0; m < nm; ++m) {
        const int k = b->member_slot[m];
        lbm_solver* h = b->slots[k];
        const int64_t bad = (int64_t)b->h_rout[2 * m + 1];
        if (r) r[k] = h->snap_valid ? b->h_rout[2 * m] : INFINITY;
        if (nonfinite) nonfinite[k] = bad;
        h->snap_valid = true;
        if (bad) worst = LBM_ERR_UNSTABLE;
    }
    if (worst != LBM_OK) b->err = "lbm_batch_residual: non-finite values in at least one member";
    return worst;
}

}  // extern "C"
