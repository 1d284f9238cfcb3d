// lbm_capi.hip -- the C ABI (include/lbm.h): lattice object, validation,
// kernel-variant selection, time stepping, reductions, readback, checkpoint.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_device.h"
#include "lbm_internal.h"

using namespace lbmd;

// ------------------------------------------------------------------ errors
// A fixed buffer per thread: recording an error allocates nothing.
static thread_local char g_err[512];

static lbm_status set_err(lbm_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

extern "C" const char *lbm_last_error(void) { return g_err; }

// ------------------------------------------------------------------ lattice
struct lbm_lattice {
    lbm_config cfg{};
    hipStream_t stream = nullptr;
    uint8_t *d_tags = nullptr;
    double *d_wall = nullptr;       // [16][3]
    void *d_pops = nullptr;
    bool own_pops = false;
    long long n_elems = 0;          // population array elements
    long long ncell = 0;
    double *d_partials = nullptr;   // [NRED][max_tiles]
    long long max_tiles = 0;
    double *d_stage1 = nullptr;     // [NRED][kFinalizeBlocks]
    int *d_tile_tag = nullptr;      // [max_tiles][4] wave classification of the current tiling
    uint32_t *d_mask = nullptr;     // [N] neighbour masks (tagged lattices)
    double *d_series = nullptr;     // [series_cap][NRED]
    long long series_cap = 0;
    void *d_mlp = nullptr;          // packed closure block (lbm_mlp.hip)
    MlpDev mlp{};
    bool has_mlp = false;
    long long t = 0;                // time counter
    int parity = 0;                 // layout parity (0: natural)
    int ms = MS_BGK;                // compiled model set
    bool tagged = true;
    int uniform_tag = LBM_TAG_BGK;
    int tx_log2 = 8;
    bool brick = false;             // brick storage layout (see Layout)
    bool pair = false;              // FP16 even step with two nodes per lane (k_collide_pair_even)
    int tiles_x = 1, tiles_y = 1, n_tiles = 1;
    long long n_fluid = 0;
    bool failed = false;
    int device = 0;                 // HIP device current at create
    char variant[96] = {0};
};

// Shared with lbm_mlp.hip.
lbm_status lbmd_fail_hip(lbm_lattice *lat, hipError_t e, const char *what) {
    if (lat) lat->failed = true;
    return set_err(LBM_EHIP, "%s: %s", what, hipGetErrorString(e));
}
lbm_status lbmd_set_err(lbm_status s, const char *msg) { return set_err(s, "%s", msg); }

#define HIPCHK(lat, expr)                                              \
    do {                                                               \
        hipError_t e_ = (expr);                                        \
        if (e_ != hipSuccess) return lbmd_fail_hip((lat), e_, #expr);  \
    } while (0)

#define CHECK_HANDLE(lat)                                                                    \
    do {                                                                                     \
        if (!(lat)) return set_err(LBM_EINVAL, "null lattice handle");                      \
        if ((lat)->failed) return set_err(LBM_ESTATE, "lattice handle failed earlier");     \
    } while (0)

// ------------------------------------------------------------ dispatch
namespace {
struct Launchers {
    hipError_t (*step)(const StepParams &, int, bool, int, int, hipStream_t);
    hipError_t (*init)(const AuxParams &, hipStream_t);
    hipError_t (*gather)(const AuxParams &, int, hipStream_t);
    hipError_t (*scatter)(const AuxParams &, hipStream_t);
    hipError_t (*face)(const AuxParams &, int, int, void *, hipStream_t);
};

template <int Q, int P>
Launchers make_launchers() {
    return {&launch_step<Q, P>, &launch_init<Q, P>, &launch_gather<Q, P>, &launch_scatter<Q, P>, &launch_face<Q, P>};
}

Launchers pick(int q, int prec) {
    if (q == 19) {
        if (prec == LBM_F64) return make_launchers<19, 0>();
        if (prec == LBM_F32) return make_launchers<19, 1>();
        return make_launchers<19, 2>();
    }
    if (prec == LBM_F64) return make_launchers<27, 0>();
    if (prec == LBM_F32) return make_launchers<27, 1>();
    return make_launchers<27, 2>();
}

size_t elem_bytes(int prec) { return prec == LBM_F64 ? 8 : (prec == LBM_F32 ? 4 : 2); }

// Population array elements: whole blocks of kBlockNodes nodes, Q slots each
// (the blocked layout of pop_base).
long long pop_elems(long long ncell, int q) { return (ncell + kBlockNodes - 1) / kBlockNodes * kBlockNodes * q; }

bool known_tag(int t) { return (t >= 0 && t <= 10) || (t >= 16 && t <= 31); }

// Storage sectors of 64 bytes hold 8 (FP64), 16 (FP32) or 32 (FP16) nodes.
int sector_log2(int prec) { return prec == LBM_F64 ? 3 : (prec == LBM_F32 ? 4 : 5); }

// Non-fluid nodes that share a storage sector with a fluid node (the step
// kernel's filler nodes).
long long count_fillers(const uint8_t *tags, long long N, int sector_log2) {
    const long long g = 1ll << sector_log2;
    long long count = 0;
    for (long long a = 0; a < N; a += g) {
        const long long b = a + g < N ? a + g : N;
        long long fl = 0;
        for (long long k = a; k < b; ++k) fl += (tags[k] >= 1 && tags[k] <= 10);
        if (fl) count += (b - a) - fl;
    }
    return count;
}

lbm_status validate(const lbm_config *c) {
    if (!c) return set_err(LBM_EINVAL, "null config");
    if (c->nx < 1 || c->ny < 1 || c->nz < 1)
        return set_err(LBM_EINVAL, "lattice size must be >= 1 (got %d x %d x %d)", c->nx, c->ny, c->nz);
    const long long n = (long long)c->nx * c->ny * c->nz;
    if (n >= (1LL << 31)) return set_err(LBM_EINVAL, "nx*ny*nz = %lld exceeds 2^31 - 1", n);
    if (c->q != 19 && c->q != 27) return set_err(LBM_EINVAL, "q must be 19 or 27 (got %d)", c->q);
    if (c->prec < 0 || c->prec > 2) return set_err(LBM_EINVAL, "unknown precision %d", c->prec);
    if ((c->flags & ~(LBM_FLAG_FREE_STREAM | LBM_FLAG_LAYOUT_BRICKS | LBM_FLAG_LAYOUT_ROWS)) != 0)
        return set_err(LBM_EINVAL, "unknown flags 0x%x", c->flags);
    if ((c->flags & LBM_FLAG_LAYOUT_BRICKS) && (c->flags & LBM_FLAG_LAYOUT_ROWS))
        return set_err(LBM_EINVAL, "LBM_FLAG_LAYOUT_BRICKS and LBM_FLAG_LAYOUT_ROWS exclude each other");
    if ((c->flags & LBM_FLAG_LAYOUT_BRICKS) && (c->nx % 16 || c->ny % 16 || c->nz % 16))
        return set_err(LBM_EINVAL, "the brick layout needs nx, ny, nz multiples of 16 (got %d x %d x %d)", c->nx, c->ny,
                       c->nz);
    if (!(c->rho0 > 0.0) || !std::isfinite(c->rho0)) return set_err(LBM_EINVAL, "rho0 must be > 0");
    if (!(c->tau > 0.5) || !std::isfinite(c->tau)) return set_err(LBM_EINVAL, "tau must be > 1/2 (got %g)", c->tau);
    if (!(c->trt_lambda > 0.0) || !std::isfinite(c->trt_lambda)) return set_err(LBM_EINVAL, "trt_lambda must be > 0");
    if (!(c->smag_cs >= 0.0) || !std::isfinite(c->smag_cs)) return set_err(LBM_EINVAL, "smag_cs must be >= 0");
    const double fm = std::sqrt(c->force[0] * c->force[0] + c->force[1] * c->force[1] + c->force[2] * c->force[2]);
    if (!(fm < 0.3)) return set_err(LBM_EINVAL, "|force| must be < 0.3");
    for (int k = 0; k < 16; ++k) {
        const double *u = c->wall_velocity[k];
        const double um = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        if (!(um < 0.3)) return set_err(LBM_EINVAL, "|wall_velocity[%d]| must be < 0.3", k);
    }
    return LBM_OK;
}

void choose_tiles(lbm_lattice *L, int txl) {
    if (L->brick) {
        // tiles of four listed 4^3 bricks (the brick layout's fixed tile); the
        // count is set when the list of bricks holding fluid is built
        L->tx_log2 = 4;
        L->tiles_x = L->cfg.nx / 16;
        L->tiles_y = L->cfg.ny / 4;
        L->n_tiles = L->tiles_x * L->tiles_y * (L->cfg.nz / 4);
        return;
    }
    L->tx_log2 = txl;
    const int TX = 1 << txl, TY = 256 >> txl;
    L->tiles_x = (L->cfg.nx + TX - 1) / TX;
    L->tiles_y = (L->cfg.ny + TY - 1) / TY;
    L->n_tiles = L->tiles_x * L->tiles_y * L->cfg.nz;
}

// Default tile width: the smallest padded row (ceil(nx/tx)*tx) over 64- to
// 256-wide tiles, larger tx on ties, so that a wave covers one contiguous row
// segment.  32-wide tiles (two half rows per wave: measured 1-11% slower on
// 400- and 480-wide lattices despite less padding) only when 64-wide ones
// would pad the row by more than a quarter.
int default_txl(int nx) {
    auto pad = [&](int l) { return (long long)((nx + (1 << l) - 1) >> l) << l; };
    int best = 8;
    for (int l = 7; l >= 6; --l)
        if (pad(l) < pad(best)) best = l;
    if (pad(6) * 4 > 5LL * nx && pad(5) < pad(best)) best = 5;
    return best;
}

StepParams step_params(const lbm_lattice *L) {
    StepParams p{};
    const lbm_config &c = L->cfg;
    p.pops = L->d_pops;
    p.tags = L->d_tags;
    p.tile_tag = L->d_tile_tag;
    p.wall_u = L->d_wall;
    p.partials = L->d_partials;
    p.partial_stride = L->max_tiles;
    p.nx = c.nx;
    p.ny = c.ny;
    p.nz = c.nz;
    p.lay = make_layout(L->brick ? 1 : 0, c.nx, c.ny);
    p.tiles_x = L->tiles_x;
    p.tiles_y = L->tiles_y;
    p.n_tiles = L->n_tiles;
    p.tiles_per_xcd = (L->n_tiles + 7) / 8;
    p.tx_log2 = L->tx_log2;
    // Row-form addressing where it pays: FP16 storage, and in FP32/FP64 the
    // wall waves of tagged lattices that are mostly fluid (measured: a
    // walled cavity gains, a porous medium with 80% solid loses).  Needs
    // whole rows per 4096-node block (nx a power of two, 64..4096) and a tile
    // at least 64 nodes wide, so that every wave lies in one row of one block.
    const long long n_nodes = (long long)c.nx * c.ny * c.nz;
    const bool rows_pay = c.prec == LBM_F16S || (L->tagged && 2 * L->n_fluid >= n_nodes);
    p.row_log2 = -1;
    if (rows_pay && !L->brick && (L->pair || L->tx_log2 >= 6) && c.nx >= 64 && c.nx <= (int)kBlockNodes &&
        (c.nx & (c.nx - 1)) == 0) {
        int l = 0;
        while ((c.nx << l) < (int)kBlockNodes) ++l;
        p.row_log2 = l;
    }
    p.pair = L->pair ? 1 : 0;
    p.n_segs = L->pair ? (int)(n_nodes / 128) : 0;
    p.mask = L->d_mask;
    p.uniform_tag = L->uniform_tag;
    p.has_force = (c.force[0] != 0.0 || c.force[1] != 0.0 || c.force[2] != 0.0) ? 1 : 0;
    p.has_mlp = L->has_mlp ? 1 : 0;
    p.rho0 = c.rho0;
    p.tau = c.tau;
    p.omega = 1.0 / c.tau;
    p.omega_minus = 1.0 / (0.5 + c.trt_lambda / (c.tau - 0.5));
    p.smag_c = 18.0 * std::sqrt(2.0) * c.smag_cs * c.smag_cs;
    p.nu0 = (c.tau - 0.5) / 3.0;
    for (int a = 0; a < 3; ++a) p.force[a] = c.force[a];
    for (int a = 0; a < 3; ++a) p.bc_u[a] = c.bc_velocity[a];
    p.bc_rho[0] = c.bc_density[0];
    p.bc_rho[1] = c.bc_density[1];
    p.mlp = L->mlp;
    return p;
}

// Variant name: lattice, precision, model set, geometry, and "/rows" when the
// step kernels use row-form addressing (depends on the tile shape).
void name_variant(lbm_lattice *L) {
    static const char *msname[] = {"bgk", "trt", "reg", "rr", "bgk+smag", "trt+open", "bgk+smag+mlp", "all"};
    const char *ms = "stream";
    for (int k = 0; k < kNumModelSets; ++k)
        if (kModelSets[k] == L->ms) ms = msname[k];
    const lbm_config &c = L->cfg;
    snprintf(L->variant, sizeof L->variant, "D3Q%d/%s/%s/%s%s", c.q,
             c.prec == LBM_F64 ? "f64" : (c.prec == LBM_F32 ? "f32" : "f16s"), ms,
             L->tagged ? "tagged" : "uniform",
             L->brick ? "/bricks" : (L->pair ? "/pairs" : (step_params(L).row_log2 >= 0 ? "/rows" : "")));
}

AuxParams aux_params(const lbm_lattice *L) {
    AuxParams a{};
    a.pops = L->d_pops;
    a.tags = L->d_tags;
    a.nx = L->cfg.nx;
    a.ny = L->cfg.ny;
    a.nz = L->cfg.nz;
    a.lay = make_layout(L->brick ? 1 : 0, L->cfg.nx, L->cfg.ny);
    a.parity = L->parity;
    a.rho0 = L->cfg.rho0;
    for (int k = 0; k < 3; ++k) a.force[k] = L->cfg.force[k];
    return a;
}

// Nodes per staging chunk: whole z-planes, at most ~256 MB of doubles.
long long chunk_cells(const lbm_lattice *L, int per_cell_doubles) {
    const long long plane = (long long)L->cfg.nx * L->cfg.ny;
    const long long cap = std::max(1LL, (256LL << 20) / (8LL * per_cell_doubles) / plane);
    return std::min<long long>(cap, L->cfg.nz) * plane;
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};
}  // namespace

// ---------------------------------------------------------- finalize kernel
namespace lbmd {
__device__ __forceinline__ void neumaier_add(double &sum, double &comp, double v) {
    const double u = sum + v;
    comp += (fabs(sum) >= fabs(v)) ? (sum - u) + v : (v - u) + sum;
    sum = u;
}

// Pairwise tree over 256 LDS values (fixed order); result in s[0].
__device__ __forceinline__ void lds_tree(double *s) {
    const int t = threadIdx.x;
    for (int w = 128; w > 0; w >>= 1) {
        __syncthreads();
        if (t < w) s[t] += s[t + w];
    }
    __syncthreads();
}

// Stage 1: block b sums a contiguous run of tiles per slot (coalesced reads,
// Neumaier per thread, pairwise tree across the block).
__global__ __launch_bounds__(256) void k_finalize1(const double *part, long long pstride, int nt, int chunk,
                                                   double *stage1) {
    __shared__ double s[256];
    const int t = threadIdx.x, b = blockIdx.x;
    const int t0 = b * chunk, t1 = min(nt, t0 + chunk);
    for (int k = 0; k < NRED; ++k) {
        double sum = 0.0, comp = 0.0;
        for (int i = t0 + t; i < t1; i += 256) neumaier_add(sum, comp, part[(long long)k * pstride + i]);
        s[t] = sum + comp;
        lds_tree(s);
        if (t == 0) stage1[k * kFinalizeBlocks + b] = s[0];
    }
}

// Stage 2: one block sums the stage-1 results per slot.
__global__ __launch_bounds__(256) void k_finalize2(const double *stage1, int nb, double *out) {
    __shared__ double s[256];
    const int t = threadIdx.x;
    for (int k = 0; k < NRED; ++k) {
        s[t] = t < nb ? stage1[k * kFinalizeBlocks + t] : 0.0;
        lds_tree(s);
        if (t == 0) out[k] = s[0];
    }
}

// Row layout.  One block per tile; wave w of the block classifies the 64 nodes
// that wave w of the step kernel updates: their fluid tag when they and their
// one-node halo (periodic) all carry that one tag, else -1 when none of them
// is fluid or a filler (every mask zero), else 0.
__global__ __launch_bounds__(256) void k_tile_classify(StepParams p, int *out) {
    const int L = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int tix = L % p.tiles_x, rem = L / p.tiles_x;
    const int tiy = rem % p.tiles_y;
    const int txl = p.tx_log2;
    const int TX = 1 << txl;
    const int z = rem / p.tiles_y;
    const int x0 = tix * TX, y0 = tiy * (256 >> txl);
    const int t = threadIdx.x;
    const int x = x0 + (t & (TX - 1)), y = y0 + (t >> txl);
    const bool in = x < p.nx && y < p.ny;
    const int xc = in ? x : x0 < p.nx ? x0 : 0, yc = in ? y : y0 < p.ny ? y0 : 0;
    const long long own = ((long long)z * p.ny + yc) * p.nx + xc;
    const int first = p.tags[own];
    const bool none = __ballot(in && p.mask[own] != 0u) == 0ull;
    // the wave's first in-range node sets the reference tag
    const unsigned long long act = __ballot(in);
    const int src = act ? __ffsll((long long)act) - 1 : 0;
    const int ref = __shfl(first, src, 64);
    bool same = act != 0ull && is_fluid_tag(ref);
    if (in) {
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int gx = (x + dx + p.nx) % p.nx, gy = (y + dy + p.ny) % p.ny;
                    const int gz = (z + dz + p.nz) % p.nz;
                    if (p.tags[((long long)gz * p.ny + gy) * p.nx + gx] != ref) same = false;
                }
    }
    // a wave is plain when every in-range lane saw only the reference tag
    const bool all = __ballot(in && !same) == 0ull && same;
    if (lane == 0) out[(long long)L * 4 + w] = all ? ref : (none ? -1 : 0);
}

hipError_t launch_tile_classify(const StepParams &p, int *out, hipStream_t s) {
    k_tile_classify<<<p.n_tiles, 256, 0, s>>>(p, out);
    return hipGetLastError();
}

// Enstrophy partials: one block per 256 nodes, |curl u|^2 / 2 with the
// eighth-order centred difference on the periodic lattice; slot 0 of the
// reduction layout holds the sum, the other slots are zero.
__device__ __forceinline__ double d8(const double *u, long long base, long long stride, int c, int n) {
    auto at = [&](int k) { return u[base + (long long)(((c + k) % n + n) % n) * stride]; };
    return 0.8 * (at(1) - at(-1)) - 0.2 * (at(2) - at(-2)) + (4.0 / 105.0) * (at(3) - at(-3)) -
           (1.0 / 280.0) * (at(4) - at(-4));
}

__global__ __launch_bounds__(256) void k_enstrophy(const double *fields, int nx, int ny, int nz, double *partials,
                                                   long long pstride) {
    const long long N = (long long)nx * ny * nz;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    double v = 0.0;
    if (t < N) {
        const int x = (int)(t % nx), y = (int)((t / nx) % ny), z = (int)(t / ((long long)nx * ny));
        const double *ux = fields + N, *uy = fields + 2 * N, *uz = fields + 3 * N;
        const long long rx = t - x, ry = t - (long long)y * nx, rz = t - (long long)z * nx * ny;
        const long long sy = nx, sz = (long long)nx * ny;
        const double wx = d8(uz, ry, sy, y, ny) - d8(uy, rz, sz, z, nz);
        const double wy = d8(ux, rz, sz, z, nz) - d8(uz, rx, 1, x, nx);
        const double wz = d8(uy, rx, 1, x, nx) - d8(ux, ry, sy, y, ny);
        v = 0.5 * (wx * wx + wy * wy + wz * wz);
    }
    __shared__ double s[4];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x < NRED)
        partials[(long long)threadIdx.x * pstride + blockIdx.x] = threadIdx.x == 0 ? (s[0] + s[1]) + (s[2] + s[3]) : 0.0;
}

hipError_t launch_finalize(const double *partials, long long partial_stride, int n_tiles, double *stage1, double *out,
                           hipStream_t s) {
    const int nb = std::min(kFinalizeBlocks, std::max(1, (n_tiles + 255) / 256));
    const int chunk = (n_tiles + nb - 1) / nb;
    k_finalize1<<<nb, 256, 0, s>>>(partials, partial_stride, n_tiles, chunk, stage1);
    k_finalize2<<<1, 256, 0, s>>>(stage1, nb, out);
    return hipGetLastError();
}
}  // namespace lbmd

// ------------------------------------------------------------------ create
extern "C" size_t lbm_population_bytes(const lbm_config *cfg) {
    if (validate(cfg) != LBM_OK) return 0;
    const long long n = (long long)cfg->nx * cfg->ny * cfg->nz;
    return (size_t)pop_elems(n, cfg->q) * elem_bytes(cfg->prec);
}

static lbm_status create_impl(const lbm_config *cfg, const uint8_t *tags_host, void *pops_dev, size_t pops_bytes,
                              void *stream, lbm_lattice **out) {
    if (!out) return set_err(LBM_EINVAL, "null output handle");
    *out = nullptr;
    lbm_status s = validate(cfg);
    if (s != LBM_OK) return s;
    if (!tags_host) return set_err(LBM_EINVAL, "null tags");
    const long long N = (long long)cfg->nx * cfg->ny * cfg->nz;

    // Tag histogram: validity, fluid count, model set, geometry.
    long long hist[32] = {0};
    for (long long n = 0; n < N; ++n) {
        const int t = tags_host[n];
        if (!known_tag(t)) return set_err(LBM_EINVAL, "unknown tag value %d at node %lld", t, n);
        if ((t == LBM_TAG_VEL_IN || t == LBM_TAG_PRES_IN) && n % cfg->nx != 0)
            return set_err(LBM_EINVAL, "open-boundary tag %d off the x = 0 plane at node %lld", t, n);
        if ((t == LBM_TAG_PRES_OUT || t == LBM_TAG_VEL_OUT) && n % cfg->nx != cfg->nx - 1)
            return set_err(LBM_EINVAL, "open-boundary tag %d off the x = nx-1 plane at node %lld", t, n);
        hist[t]++;
    }
    const long long n_open = hist[LBM_TAG_VEL_IN] + hist[LBM_TAG_PRES_OUT] + hist[LBM_TAG_PRES_IN] + hist[LBM_TAG_VEL_OUT];
    if (n_open && cfg->nx < 2) return set_err(LBM_EINVAL, "open boundaries need nx >= 2");
    if (hist[LBM_TAG_VEL_IN] || hist[LBM_TAG_VEL_OUT]) {
        const double *u = cfg->bc_velocity;
        if (!(std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) < 0.3))
            return set_err(LBM_EINVAL, "|bc_velocity| must be < 0.3");
    }
    if (hist[LBM_TAG_PRES_IN] && !(cfg->bc_density[0] > 0.0)) return set_err(LBM_EINVAL, "bc_density[0] must be > 0");
    if (hist[LBM_TAG_PRES_OUT] && !(cfg->bc_density[1] > 0.0)) return set_err(LBM_EINVAL, "bc_density[1] must be > 0");
    long long nf = 0;
    for (int t = 1; t <= 10; ++t) nf += hist[t];
    if (nf == 0) return set_err(LBM_EINVAL, "no fluid node");
    int need = 0;
    if (hist[LBM_TAG_BGK]) need |= MS_BGK;
    if (hist[LBM_TAG_TRT]) need |= MS_TRT;
    if (hist[LBM_TAG_BGK_SMAG]) need |= MS_SMAG;
    if (hist[LBM_TAG_BGK_MLP]) need |= MS_MLP;
    if (hist[LBM_TAG_REG]) need |= MS_REG;
    if (n_open) need |= MS_OPEN;
    if (hist[LBM_TAG_RR]) need |= MS_RR;
    int ms = -1;
    for (int k = 0; k < kNumModelSets; ++k)
        if ((kModelSets[k] & need) == need) {
            ms = kModelSets[k];
            break;
        }
    if (ms < 0) return set_err(LBM_EUNSUPPORTED, "no compiled model set covers the tags");
    if (cfg->flags & LBM_FLAG_FREE_STREAM) ms = MS_STREAM;
    int n_models = 0, only = LBM_TAG_BGK;
    for (int t = 1; t <= 10; ++t)
        if (hist[t]) {
            n_models++;
            only = t;
        }
    const bool one_model = nf == N && n_models == 1;
    // Brick layout: on request, or by default for solid-rich tagged lattices
    // (fewer than half the nodes fluid) whose sides are multiples of 16: there
    // the 4 x 4 x 1 sectors of the brick order hold fluid far more often than
    // the 16-node row segments of the row order.
    const bool dims16 = cfg->nx % 16 == 0 && cfg->ny % 16 == 0 && cfg->nz % 16 == 0;
    const bool brick = (cfg->flags & LBM_FLAG_LAYOUT_BRICKS) ||
                       (!(cfg->flags & LBM_FLAG_LAYOUT_ROWS) && dims16 && !one_model && 2 * nf < N);
    // Lattices of one fluid model without walls run the untagged kernels
    // (no tags or masks read), unless they take the brick layout, which only
    // the tagged kernels implement.
    const bool tagged = !one_model || brick;
    // Odd-step filler stores pay off where filler nodes are few (walls of a
    // mostly fluid domain); in solid-rich media (porous rock) they add more
    // scattered partial writes than they complete, so there only the even
    // step fills.
    const bool odd_fill = tagged && !brick && count_fillers(tags_host, N, sector_log2(cfg->prec)) * 16 <= nf;

    const size_t need_bytes = lbm_population_bytes(cfg);
    if (pops_dev) {
        if (pops_bytes < need_bytes)
            return set_err(LBM_EINVAL, "population buffer has %zu bytes, needs %zu", pops_bytes, need_bytes);
        if (reinterpret_cast<uintptr_t>(pops_dev) % 256 != 0)
            return set_err(LBM_EINVAL, "population buffer must be 256-byte aligned");
    }

    lbm_lattice *L = new (std::nothrow) lbm_lattice();
    if (!L) return set_err(LBM_ENOMEM, "host allocation failed");
    L->cfg = *cfg;
    L->stream = static_cast<hipStream_t>(stream);
    L->ncell = N;
    L->n_elems = pop_elems(N, cfg->q);
    L->n_fluid = nf;
    L->ms = ms;
    L->tagged = tagged;
    L->uniform_tag = only;
    L->brick = brick;
    // FP16 lattices of one model without walls whose rows tile the 4096-node
    // blocks and hold whole 128-node segments: even steps with two nodes per lane
    L->pair = cfg->prec == LBM_F16S && !tagged && (ms & MS_MLP) == 0 && cfg->nx >= 128 &&
              cfg->nx <= (int)kBlockNodes && (cfg->nx & (cfg->nx - 1)) == 0;
    choose_tiles(L, default_txl(cfg->nx));
    name_variant(L);

    auto bail = [&](lbm_status st) {
        lbm_destroy(L);
        return st;
    };
    hipError_t e = hipGetDevice(&L->device);
    if (e != hipSuccess) return bail(set_err(LBM_EHIP, "hipGetDevice: %s", hipGetErrorString(e)));
    if (pops_dev) {
        L->d_pops = pops_dev;
        L->own_pops = false;
    } else {
        e = hipMalloc(&L->d_pops, need_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            L->d_pops = nullptr;
            return bail(set_err(LBM_ENOMEM, "hipMalloc of %zu population bytes failed: %s", need_bytes,
                                hipGetErrorString(e)));
        }
        L->own_pops = true;
    }
    e = hipMalloc(&L->d_tags, (size_t)N);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        L->d_tags = nullptr;
        return bail(set_err(LBM_ENOMEM, "hipMalloc of tags failed"));
    }
    e = hipMalloc(&L->d_wall, 16 * 3 * sizeof(double));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        L->d_wall = nullptr;
        return bail(set_err(LBM_ENOMEM, "hipMalloc of wall table failed"));
    }
    // Partials sized for the tiling with the most tiles over every allowed tile width.
    long long max_tiles = 0;
    for (int l = 5; l <= 8; ++l) {
        const long long tx = 1LL << l, ty = 256 >> l;
        max_tiles = std::max(max_tiles, ((cfg->nx + tx - 1) / tx) * ((cfg->ny + ty - 1) / ty) * cfg->nz);
    }
    L->max_tiles = max_tiles;
    e = hipMalloc(&L->d_partials, (size_t)max_tiles * NRED * sizeof(double));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        L->d_partials = nullptr;
        return bail(set_err(LBM_ENOMEM, "hipMalloc of reduction partials failed"));
    }
    e = hipMalloc(&L->d_stage1, (size_t)kFinalizeBlocks * NRED * sizeof(double));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        L->d_stage1 = nullptr;
        return bail(set_err(LBM_ENOMEM, "hipMalloc of reduction stage buffer failed"));
    }
    e = hipMalloc(&L->d_tile_tag, (size_t)max_tiles * 4 * sizeof(int));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        L->d_tile_tag = nullptr;
        return bail(set_err(LBM_ENOMEM, "hipMalloc of tile classes failed"));
    }
    if (tagged) {
        e = hipMalloc(&L->d_mask, (size_t)N * sizeof(uint32_t));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            L->d_mask = nullptr;
            return bail(set_err(LBM_ENOMEM, "hipMalloc of neighbour masks failed"));
        }
    }
    // tags on the device in storage order
    const Layout lay = make_layout(brick ? 1 : 0, cfg->nx, cfg->ny);
    std::vector<uint8_t> stags;
    std::vector<int> blist;
    const uint8_t *up = tags_host;
    if (brick) {
        try {
            stags.resize((size_t)N);
        } catch (...) {
            return bail(set_err(LBM_ENOMEM, "host allocation failed"));
        }
        for (int z = 0; z < cfg->nz; ++z)
            for (int y = 0; y < cfg->ny; ++y) {
                const uint8_t *row = tags_host + ((long long)z * cfg->ny + y) * cfg->nx;
                const int base = lay.z(z) + lay.y(y);
                for (int x = 0; x < cfg->nx; ++x) stags[(size_t)(base + lay.x(x))] = row[x];
            }
        up = stags.data();
        // The bricks that hold fluid, in storage order (bricks are 64 consecutive
        // storage indices), four to a tile, -1 padding the last tile.  A brick
        // without fluid has no filler either (its sectors hold no fluid), so no
        // wave is launched for it.
        try {
            blist.reserve((size_t)(N / 64) + 4);
        } catch (...) {
            return bail(set_err(LBM_ENOMEM, "host allocation failed"));
        }
        for (long long b = 0; b < N / 64; ++b) {
            bool any = false;
            for (int k = 0; k < 64 && !any; ++k) any = is_fluid_tag(stags[(size_t)(b * 64 + k)]);
            if (any) blist.push_back((int)b);
        }
        while (blist.size() % 4) blist.push_back(-1);
        L->n_tiles = (int)(blist.size() / 4);
    }
    e = hipMemcpyAsync(L->d_tags, up, (size_t)N, hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(L->d_wall, cfg->wall_velocity, 16 * 3 * sizeof(double), hipMemcpyHostToDevice, L->stream);
    if (e == hipSuccess && L->tagged)
        e = cfg->q == 19 ? launch_build_mask<19>(L->d_tags, cfg->nx, cfg->ny, cfg->nz, lay, sector_log2(cfg->prec),
                                                 odd_fill, L->d_mask, L->stream)
                         : launch_build_mask<27>(L->d_tags, cfg->nx, cfg->ny, cfg->nz, lay, sector_log2(cfg->prec),
                                                 odd_fill, L->d_mask, L->stream);
    // wave classes (from the tags and the masks just built), or the brick list
    if (e == hipSuccess && L->tagged) {
        if (brick)
            e = hipMemcpyAsync(L->d_tile_tag, blist.data(), blist.size() * sizeof(int), hipMemcpyHostToDevice,
                               L->stream);
        else
            e = launch_tile_classify(step_params(L), L->d_tile_tag, L->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) return bail(lbmd_fail_hip(nullptr, e, "tag upload"));
    if (brick) std::vector<uint8_t>().swap(stags);
    if (e == hipSuccess) e = hipStreamSynchronize(L->stream);
    if (e != hipSuccess) return bail(lbmd_fail_hip(nullptr, e, "tag upload"));
    *out = L;
    return LBM_OK;
}

extern "C" lbm_status lbm_create(const lbm_config *cfg, const uint8_t *tags_host, void *hip_stream,
                                 lbm_lattice **out) {
    return create_impl(cfg, tags_host, nullptr, 0, hip_stream, out);
}

extern "C" lbm_status lbm_create_on_buffer(const lbm_config *cfg, const uint8_t *tags_host, void *pops_dev,
                                           size_t pops_bytes, void *hip_stream, lbm_lattice **out) {
    if (!pops_dev) return set_err(LBM_EINVAL, "null population buffer");
    return create_impl(cfg, tags_host, pops_dev, pops_bytes, hip_stream, out);
}

void lbmd_free_mlp(lbm_lattice *lat);  // lbm_mlp.hip

extern "C" void lbm_destroy(lbm_lattice *lat) {
    if (!lat) return;
    if (lat->stream || lat->d_pops) (void)hipStreamSynchronize(lat->stream);
    if (lat->own_pops && lat->d_pops) (void)hipFree(lat->d_pops);
    if (lat->d_tags) (void)hipFree(lat->d_tags);
    if (lat->d_wall) (void)hipFree(lat->d_wall);
    if (lat->d_partials) (void)hipFree(lat->d_partials);
    if (lat->d_stage1) (void)hipFree(lat->d_stage1);
    if (lat->d_tile_tag) (void)hipFree(lat->d_tile_tag);
    if (lat->d_mask) (void)hipFree(lat->d_mask);
    if (lat->d_series) (void)hipFree(lat->d_series);
    lbmd_free_mlp(lat);
    delete lat;
}

extern "C" lbm_status lbm_set_launch(lbm_lattice *lat, int tx, int ty) {
    CHECK_HANDLE(lat);
    if (lat->brick) return set_err(LBM_EUNSUPPORTED, "the brick layout has a fixed 16 x 4 x 4 tile");
    int l = -1;
    for (int k = 5; k <= 8; ++k)
        if (tx == (1 << k)) l = k;
    if (l < 0 || tx * ty != 256) return set_err(LBM_EINVAL, "tile must be tx in {32,64,128,256} with tx*ty = 256");
    lat->pair = false;  // an explicit tile selects the one-node kernels
    choose_tiles(lat, l);
    name_variant(lat);
    if (lat->tagged) HIPCHK(lat, launch_tile_classify(step_params(lat), lat->d_tile_tag, lat->stream));
    return LBM_OK;
}

extern "C" const char *lbm_variant_name(const lbm_lattice *lat) { return lat ? lat->variant : ""; }

extern "C" int64_t lbm_time(const lbm_lattice *lat) { return lat ? lat->t : -1; }

extern "C" lbm_status lbm_synchronize(lbm_lattice *lat) {
    CHECK_HANDLE(lat);
    HIPCHK(lat, hipStreamSynchronize(lat->stream));
    return LBM_OK;
}

extern "C" int lbm_velocity(int q, int i, int c[3], double *w) {
    if ((q != 19 && q != 27) || i < 0 || i >= q || !c || !w) return -1;
    // The device tables are compile-time; mirror them through a small host loop.
    int out = -1;
    auto fill = [&](auto I) {
        constexpr int k = decltype(I)::value;
        if (k == i) {
            if (q == 19) {
                if constexpr (k < 19) {
                    using Vk = V<19, k>;
                    c[0] = Vk::x, c[1] = Vk::y, c[2] = Vk::z, *w = Vk::w, out = Vk::opp;
                }
            } else {
                using Vk = V<27, k>;
                c[0] = Vk::x, c[1] = Vk::y, c[2] = Vk::z, *w = Vk::w, out = Vk::opp;
            }
        }
    };
    [&]<int... Is>(std::integer_sequence<int, Is...>) { (fill(std::integral_constant<int, Is>{}), ...); }(
        std::make_integer_sequence<int, 27>{});
    return out;
}

// ------------------------------------------------------------ initial state
extern "C" lbm_status lbm_init_equilibrium(lbm_lattice *lat, const double *rho_host, const double *u_host) {
    CHECK_HANDLE(lat);
    const long long N = lat->ncell;
    const long long chunk = chunk_cells(lat, 4);
    DevBuf buf;
    HIPCHK(lat, hipMalloc(&buf.p, (size_t)chunk * 4 * sizeof(double)));
    double *d = static_cast<double *>(buf.p);
    const Launchers Lc = pick(lat->cfg.q, lat->cfg.prec);
    for (long long c0 = 0; c0 < N; c0 += chunk) {
        const long long cnt = std::min(chunk, N - c0);
        AuxParams a = aux_params(lat);
        a.cell0 = c0;
        a.count = cnt;
        a.in_rho = nullptr;
        a.in_u = nullptr;
        if (rho_host) {
            HIPCHK(lat, hipMemcpyAsync(d, rho_host + c0, cnt * sizeof(double), hipMemcpyHostToDevice, lat->stream));
            a.in_rho = d;
        }
        if (u_host) {
            for (int k = 0; k < 3; ++k)
                HIPCHK(lat, hipMemcpyAsync(d + (1 + k) * cnt, u_host + k * N + c0, cnt * sizeof(double),
                                           hipMemcpyHostToDevice, lat->stream));
            a.in_u = d + cnt;
        }
        HIPCHK(lat, Lc.init(a, lat->stream));
        HIPCHK(lat, hipStreamSynchronize(lat->stream));
    }
    lat->t = 0;
    lat->parity = 0;
    return LBM_OK;
}

// --------------------------------------------------------------- stepping
// partials: where MODE_STEP_REDUCE / MODE_REDUCE write the per-tile sums
// ([NRED][stride]); null = the lattice's own buffer.
static lbm_status launch_one(lbm_lattice *lat, int mode, double *partials = nullptr, long long stride = 0) {
    const Launchers Lc = pick(lat->cfg.q, lat->cfg.prec);
    StepParams p = step_params(lat);
    if (partials) {
        p.partials = partials;
        p.partial_stride = stride;
    }
    HIPCHK(lat, Lc.step(p, lat->ms, lat->tagged, mode, lat->parity, lat->stream));
    if (mode != MODE_REDUCE) {
        lat->parity ^= 1;
        lat->t += 1;
    }
    return LBM_OK;
}

extern "C" lbm_status lbm_step(lbm_lattice *lat, int64_t n_steps) {
    CHECK_HANDLE(lat);
    if (n_steps < 0) return set_err(LBM_EINVAL, "n_steps must be >= 0");
    for (int64_t s = 0; s < n_steps; ++s) {
        lbm_status st = launch_one(lat, MODE_STEP);
        if (st != LBM_OK) return st;
    }
    return LBM_OK;
}

static lbm_status ensure_series(lbm_lattice *lat, long long n) {
    if (n <= lat->series_cap) return LBM_OK;
    if (lat->d_series) {
        HIPCHK(lat, hipStreamSynchronize(lat->stream));
        HIPCHK(lat, hipFree(lat->d_series));
        lat->d_series = nullptr;
    }
    HIPCHK(lat, hipMalloc(&lat->d_series, (size_t)n * NRED * sizeof(double)));
    lat->series_cap = n;
    return LBM_OK;
}

static void fill_moments(const lbm_lattice *lat, const double *v, int64_t step, lbm_moments *m) {
    m->step = step;
    m->n_fluid = lat->n_fluid;
    m->n_nonfinite = (int64_t)std::llround(v[9]);
    m->mass_delta = v[0];
    m->mass = (double)lat->n_fluid * lat->cfg.rho0 + v[0];
    for (int a = 0; a < 3; ++a) {
        m->momentum[a] = v[1 + a];
        m->velocity_sum[a] = v[4 + a];
    }
    m->kinetic_energy = v[7] / (double)lat->n_fluid;
    m->kinetic_energy_rho = v[8];
}

// Shared by lbm_step_reduce and lbm_step_reduce_noalloc: the step loop with
// fused reductions every `every` steps into partials ([NRED][stride]), the
// two-stage finalize through stage1 into d_series ([ns][NRED]), and the copy
// of the samples to the host through a fixed stack buffer.
static lbm_status step_reduce_impl(lbm_lattice *lat, int64_t n_steps, int64_t every, lbm_moments *series,
                                   double *partials, long long stride, double *stage1, double *d_series) {
    const int64_t ns = n_steps / every + 1;
    const int64_t t0 = lat->t;
    lbm_status st;
    for (int64_t s = 0; s < n_steps; ++s) {
        if (s % every == 0) {
            st = launch_one(lat, MODE_STEP_REDUCE, partials, stride);
            if (st != LBM_OK) return st;
            HIPCHK(lat, launch_finalize(partials, stride, lat->n_tiles, stage1, d_series + (s / every) * NRED,
                                        lat->stream));
        } else {
            st = launch_one(lat, MODE_STEP);
            if (st != LBM_OK) return st;
        }
    }
    if (n_steps % every == 0) {
        st = launch_one(lat, MODE_REDUCE, partials, stride);
        if (st != LBM_OK) return st;
        HIPCHK(lat, launch_finalize(partials, stride, lat->n_tiles, stage1, d_series + (ns - 1) * NRED, lat->stream));
    }
    constexpr int64_t kBatch = 64;
    double h[kBatch * NRED];
    bool bad = false;
    for (int64_t k0 = 0; k0 < ns; k0 += kBatch) {
        const int64_t cnt = std::min(kBatch, ns - k0);
        HIPCHK(lat, hipMemcpyAsync(h, d_series + k0 * NRED, (size_t)cnt * NRED * sizeof(double),
                                   hipMemcpyDeviceToHost, lat->stream));
        HIPCHK(lat, hipStreamSynchronize(lat->stream));
        for (int64_t k = 0; k < cnt; ++k) {
            fill_moments(lat, h + k * NRED, t0 + (k0 + k) * every, &series[k0 + k]);
            if (series[k0 + k].n_nonfinite > 0) bad = true;
        }
    }
    if (bad) return set_err(LBM_EUNSTABLE, "non-finite density or velocity found");
    return LBM_OK;
}

extern "C" lbm_status lbm_step_reduce(lbm_lattice *lat, int64_t n_steps, int64_t every, lbm_moments *series,
                                      int64_t n_series) {
    CHECK_HANDLE(lat);
    if (n_steps < 0 || every < 1) return set_err(LBM_EINVAL, "need n_steps >= 0 and every >= 1");
    const int64_t ns = n_steps / every + 1;
    if (!series || n_series < ns) return set_err(LBM_EINVAL, "series needs %lld entries", (long long)ns);
    lbm_status st = ensure_series(lat, ns);
    if (st != LBM_OK) return st;
    return step_reduce_impl(lat, n_steps, every, series, lat->d_partials, lat->max_tiles, lat->d_stage1,
                            lat->d_series);
}

// ------------------------------------------- allocation-free step + reduce
// The reduction scratch of lbm_step_reduce_noalloc: per-tile partials, the
// finalize stage and the sample series, in one array per GPU that lives as
// long as the process.  In host code `scratch` only names the symbol; its
// device address comes from hipGetSymbolAddress, once per device.
namespace {
constexpr long long kNoAllocTiles = LBM_NOALLOC_MAX_TILES;
constexpr long long kNoAllocSamples = LBM_NOALLOC_MAX_SAMPLES;
constexpr long long kScratchDoubles = NRED * kNoAllocTiles + NRED * kFinalizeBlocks + NRED * kNoAllocSamples;
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `dev` (resolved with dev current, then cached).
lbm_status scratch_on(int dev, double **out) {
    if (dev < 0 || dev >= kMaxDevices) return set_err(LBM_EUNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
        void *ptr = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr)
            return set_err(LBM_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}
}  // namespace

extern "C" lbm_status lbm_step_reduce_noalloc(lbm_lattice *lat, int64_t n_steps, int64_t every,
                                              lbm_moments *series, int64_t n_series) {
    CHECK_HANDLE(lat);
    if (n_steps < 0 || every < 1) return set_err(LBM_EINVAL, "need n_steps >= 0 and every >= 1");
    const int64_t ns = n_steps / every + 1;
    if (!series || n_series < ns) return set_err(LBM_EINVAL, "series needs %lld entries", (long long)ns);
    if (ns > kNoAllocSamples)
        return set_err(LBM_EINVAL, "%lld samples exceed the allocation-free limit of %lld", (long long)ns,
                       kNoAllocSamples);
    if (lat->n_tiles > kNoAllocTiles)
        return set_err(LBM_EINVAL, "%d tiles exceed the allocation-free limit of %lld (about %lld nodes)",
                       lat->n_tiles, kNoAllocTiles, kNoAllocTiles * 256);
    double *base = nullptr;
    lbm_status st = scratch_on(lat->device, &base);
    if (st != LBM_OK) return st;
    double *partials = base;
    double *stage1 = base + NRED * kNoAllocTiles;
    double *d_series = stage1 + NRED * kFinalizeBlocks;
    return step_reduce_impl(lat, n_steps, every, series, partials, kNoAllocTiles, stage1, d_series);
}

extern "C" lbm_status lbm_reduce(lbm_lattice *lat, lbm_moments *out) {
    CHECK_HANDLE(lat);
    if (!out) return set_err(LBM_EINVAL, "null output");
    return lbm_step_reduce(lat, 0, 1, out, 1);
}

// ---------------------------------------------------------------- readback
static lbm_status gather_range(lbm_lattice *lat, int gmode, double *host, int per_cell, int shifted) {
    const long long N = lat->ncell;
    const long long chunk = chunk_cells(lat, per_cell);
    DevBuf buf;
    HIPCHK(lat, hipMalloc(&buf.p, (size_t)chunk * per_cell * sizeof(double)));
    double *d = static_cast<double *>(buf.p);
    const Launchers Lc = pick(lat->cfg.q, lat->cfg.prec);
    for (long long c0 = 0; c0 < N; c0 += chunk) {
        const long long cnt = std::min(chunk, N - c0);
        AuxParams a = aux_params(lat);
        a.cell0 = c0;
        a.count = cnt;
        a.out = d;
        a.shifted = shifted;
        HIPCHK(lat, Lc.gather(a, gmode, lat->stream));
        for (int k = 0; k < per_cell; ++k)
            HIPCHK(lat, hipMemcpyAsync(host + k * N + c0, d + k * cnt, cnt * sizeof(double), hipMemcpyDeviceToHost,
                                       lat->stream));
        HIPCHK(lat, hipStreamSynchronize(lat->stream));
    }
    return LBM_OK;
}

extern "C" lbm_status lbm_read_fields(lbm_lattice *lat, double *rho_host, double *u_host) {
    CHECK_HANDLE(lat);
    if (!rho_host && !u_host) return LBM_OK;
    const long long N = lat->ncell;
    std::vector<double> tmp;
    double *dst;
    try {
        tmp.resize((size_t)N * 4);
    } catch (...) {
        return set_err(LBM_ENOMEM, "host allocation failed");
    }
    dst = tmp.data();
    lbm_status st = gather_range(lat, G_FIELDS, dst, 4, 0);
    if (st != LBM_OK) return st;
    if (rho_host) std::memcpy(rho_host, dst, (size_t)N * sizeof(double));
    if (u_host) std::memcpy(u_host, dst + N, (size_t)N * 3 * sizeof(double));
    return LBM_OK;
}

extern "C" lbm_status lbm_read_populations(lbm_lattice *lat, double *f_host) {
    CHECK_HANDLE(lat);
    if (!f_host) return set_err(LBM_EINVAL, "null output");
    return gather_range(lat, G_POPS, f_host, lat->cfg.q, 0);
}

extern "C" lbm_status lbm_read_state(lbm_lattice *lat, double *h_host) {
    CHECK_HANDLE(lat);
    if (!h_host) return set_err(LBM_EINVAL, "null output");
    return gather_range(lat, G_POPS, h_host, lat->cfg.q, 1);
}

extern "C" lbm_status lbm_read_cells(lbm_lattice *lat, const int64_t *cells_host, int64_t n, double *f_host) {
    CHECK_HANDLE(lat);
    if (n < 0 || (n > 0 && (!cells_host || !f_host))) return set_err(LBM_EINVAL, "bad cell list");
    if (n == 0) return LBM_OK;
    for (int64_t k = 0; k < n; ++k)
        if (cells_host[k] < 0 || cells_host[k] >= lat->ncell)
            return set_err(LBM_EINVAL, "cell index %lld out of range", (long long)cells_host[k]);
    const int q = lat->cfg.q;
    DevBuf buf;
    HIPCHK(lat, hipMalloc(&buf.p, (size_t)n * (q + 1) * sizeof(double)));
    long long *dc = static_cast<long long *>(buf.p);
    double *dout = reinterpret_cast<double *>(dc + n);
    HIPCHK(lat, hipMemcpyAsync(dc, cells_host, (size_t)n * sizeof(int64_t), hipMemcpyHostToDevice, lat->stream));
    AuxParams a = aux_params(lat);
    a.cells = dc;
    a.count = n;
    a.out = dout;
    HIPCHK(lat, pick(q, lat->cfg.prec).gather(a, G_CELLS, lat->stream));
    HIPCHK(lat, hipMemcpyAsync(f_host, dout, (size_t)n * q * sizeof(double), hipMemcpyDeviceToHost, lat->stream));
    HIPCHK(lat, hipStreamSynchronize(lat->stream));
    return LBM_OK;
}

static lbm_status scatter_range(lbm_lattice *lat, const double *f_host, int64_t t, int shifted);

extern "C" lbm_status lbm_write_populations(lbm_lattice *lat, const double *f_host, int64_t t) {
    CHECK_HANDLE(lat);
    return scatter_range(lat, f_host, t, 0);
}

extern "C" lbm_status lbm_write_state(lbm_lattice *lat, const double *h_host, int64_t t) {
    CHECK_HANDLE(lat);
    return scatter_range(lat, h_host, t, 1);
}

static lbm_status scatter_range(lbm_lattice *lat, const double *f_host, int64_t t, int shifted) {
    if (!f_host) return set_err(LBM_EINVAL, "null input");
    if (t < 0) return set_err(LBM_EINVAL, "time must be >= 0");
    const int q = lat->cfg.q;
    const long long N = lat->ncell;
    const long long chunk = chunk_cells(lat, q);
    DevBuf buf;
    HIPCHK(lat, hipMalloc(&buf.p, (size_t)chunk * q * sizeof(double)));
    double *d = static_cast<double *>(buf.p);
    const Launchers Lc = pick(q, lat->cfg.prec);
    for (long long c0 = 0; c0 < N; c0 += chunk) {
        const long long cnt = std::min(chunk, N - c0);
        for (int k = 0; k < q; ++k)
            HIPCHK(lat, hipMemcpyAsync(d + k * cnt, f_host + k * N + c0, cnt * sizeof(double), hipMemcpyHostToDevice,
                                       lat->stream));
        AuxParams a = aux_params(lat);
        a.cell0 = c0;
        a.count = cnt;
        a.in_f = d;
        a.shifted = shifted;
        HIPCHK(lat, Lc.scatter(a, lat->stream));
        HIPCHK(lat, hipStreamSynchronize(lat->stream));
    }
    lat->parity = 0;
    lat->t = t;
    return LBM_OK;
}

extern "C" int lbm_face_populations(int q) { return q == 19 ? 5 : (q == 27 ? 9 : 0); }

static lbm_status face_copy(lbm_lattice *lat, int face, int unpack, void *buf) {
    CHECK_HANDLE(lat);
    if (face != 0 && face != 1) return set_err(LBM_EINVAL, "face must be 0 (z = 0) or 1 (z = nz-1)");
    if (!buf) return set_err(LBM_EINVAL, "null face buffer");
    AuxParams a = aux_params(lat);
    HIPCHK(lat, pick(lat->cfg.q, lat->cfg.prec).face(a, face, unpack, buf, lat->stream));
    return LBM_OK;
}

extern "C" lbm_status lbm_face_pack(lbm_lattice *lat, int face, void *buf_dev) {
    return face_copy(lat, face, 0, buf_dev);
}

extern "C" lbm_status lbm_face_unpack(lbm_lattice *lat, int face, const void *buf_dev) {
    return face_copy(lat, face, 1, const_cast<void *>(buf_dev));
}

extern "C" lbm_status lbm_enstrophy(lbm_lattice *lat, double *out) {
    CHECK_HANDLE(lat);
    if (!out) return set_err(LBM_EINVAL, "null output");
    const lbm_config &c = lat->cfg;
    if (lat->n_fluid != lat->ncell) return set_err(LBM_EUNSUPPORTED, "enstrophy needs an all-fluid lattice");
    if (c.nx < 9 || c.ny < 9 || c.nz < 9) return set_err(LBM_EUNSUPPORTED, "enstrophy needs every axis >= 9 nodes");
    const long long N = lat->ncell;
    const long long nblocks = (N + 255) / 256;
    DevBuf fields, part, res;
    HIPCHK(lat, hipMalloc(&fields.p, (size_t)N * 4 * sizeof(double)));
    HIPCHK(lat, hipMalloc(&part.p, (size_t)nblocks * NRED * sizeof(double)));
    HIPCHK(lat, hipMalloc(&res.p, NRED * sizeof(double)));
    AuxParams a = aux_params(lat);
    a.cell0 = 0;
    a.count = N;
    a.out = static_cast<double *>(fields.p);
    HIPCHK(lat, pick(c.q, c.prec).gather(a, G_FIELDS, lat->stream));
    k_enstrophy<<<(unsigned)nblocks, 256, 0, lat->stream>>>(static_cast<const double *>(fields.p), c.nx, c.ny, c.nz,
                                                            static_cast<double *>(part.p), nblocks);
    HIPCHK(lat, hipGetLastError());
    HIPCHK(lat, launch_finalize(static_cast<const double *>(part.p), nblocks, (int)nblocks, lat->d_stage1,
                                static_cast<double *>(res.p), lat->stream));
    double h[NRED];
    HIPCHK(lat, hipMemcpyAsync(h, res.p, sizeof h, hipMemcpyDeviceToHost, lat->stream));
    HIPCHK(lat, hipStreamSynchronize(lat->stream));
    *out = h[0] / (double)N;
    return LBM_OK;
}

// ------------------------------------------------- accessors for lbm_mlp.hip
lbm_config lbmd_config(const lbm_lattice *lat) { return lat->cfg; }
hipStream_t lbmd_stream(const lbm_lattice *lat) { return lat->stream; }
bool lbmd_failed(const lbm_lattice *lat) { return lat->failed; }
void lbmd_set_mlp(lbm_lattice *lat, void *block, const MlpDev &m) {
    lat->d_mlp = block;
    lat->mlp = m;
    lat->has_mlp = true;
}
void *lbmd_mlp_block(lbm_lattice *lat) { return lat->d_mlp; }
void lbmd_clear_mlp(lbm_lattice *lat) {
    lat->d_mlp = nullptr;
    lat->has_mlp = false;
}
// Natural-state gather of the whole lattice into device memory (FP64,
// `per_cell` = 4 fields: rho, ux, uy, uz as planes).  Used by the filter.
lbm_status lbmd_fields_device(lbm_lattice *lat, double *d_out) {
    AuxParams a = aux_params(lat);
    a.cell0 = 0;
    a.count = lat->ncell;
    a.out = d_out;
    HIPCHK(lat, pick(lat->cfg.q, lat->cfg.prec).gather(a, G_FIELDS, lat->stream));
    return LBM_OK;
}
