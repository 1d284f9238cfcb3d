// lbm_internal.h -- host/device shared declarations of the HIP library.
//
// Parameter blocks passed by value to the kernels, and the per-(Q, precision)
// launcher entry points.  Each launcher lives in its own translation unit
// (lbm_q{19,27}_{f64,f32,f16}.hip) so the kernel variants compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "lbm.h"
#include "lbm_device.h"

namespace lbmd {

// Collision-model sets a step kernel can be specialised on (the kernel-size
// reduction of Sec. 2.3: only the models present are compiled in).
enum ModelSet : int {
    MS_BGK = 1,
    MS_TRT = 2,
    MS_SMAG = 4,
    MS_MLP = 8,
    MS_REG = 16,
    MS_OPEN = 32,  // regularized velocity / pressure boundary nodes on the x planes
    MS_RR = 64,    // recursive regularized
    MS_STREAM = 128,  // no collision (LBM_FLAG_FREE_STREAM): pure streaming
};
constexpr int kAllModels = MS_BGK | MS_TRT | MS_SMAG | MS_MLP | MS_REG | MS_OPEN | MS_RR;

// Compiled model-set variants, smallest first.  The host picks the first one
// that covers the fluid tags present.
constexpr int kModelSets[] = {MS_BGK, MS_TRT, MS_REG, MS_RR, MS_BGK | MS_SMAG, MS_TRT | MS_OPEN,
                              MS_BGK | MS_SMAG | MS_MLP, kAllModels};
constexpr int kNumModelSets = 8;

// Kernel modes.
enum StepMode : int {
    MODE_STEP = 0,        // collide + stream
    MODE_STEP_REDUCE = 1, // collide + stream + reductions of the loaded state
    MODE_REDUCE = 2,      // reductions of the current state only (no stores)
};

// Reduction slots per sample: sum drho, sum rho u (3), sum u (3), sum u^2/2,
// sum rho u^2/2, count of non-finite nodes.
constexpr int NRED = 10;

// Packed closure parameters on the device: BF16 weights (as uint16 bit
// patterns) followed by FP32 biases and normalisation (see lbm_mlp.hip).
struct MlpDev {
    const uint16_t *w1;   // [32][8]: W1 rows padded from 7 to 8 inputs (zero)
    const uint16_t *w2;   // [2 products][2 lane groups][32 rows][8 K slots], columns
                          // permuted to the layer-1 accumulator order
    const uint16_t *w3;   // [2 lane groups][16]: W3 in accumulator order
    const float *b1;      // [2 lane groups][16]: b1 in accumulator order
    const float *b2;      // [2 lane groups][16]: b2 in accumulator order
    const float *b3;      // [1]
    const float *mean;    // [7]
    const float *inv_sd;  // [7] FP32 reciprocals of the standard deviations
};

struct StepParams {
    void *pops;               // population array (blocked layout, see pop_base)
    const uint8_t *tags;      // device tags (TAGGED variants)
    const int *tile_tag;      // per tile and wave ([tile][4], 32-bit words: one scalar
                              // load per wave).  Row layout: the fluid tag when the
                              // wave's 64 nodes and their one-node halo are that one
                              // model, -1 when none of its nodes is fluid or a filler
                              // (the wave has nothing to do), else 0.  Brick layout:
                              // the storage index / 64 of the wave's brick (the bricks
                              // holding fluid, in storage order), -1 past the last
    const uint32_t *mask;     // per-node neighbour mask (TAGGED variants)
    const double *wall_u;     // [16][3] moving-wall velocities (device)
    double *partials;         // [NRED][partial_stride] per-tile reduction partials
    long long partial_stride; // tiles per reduction slot in `partials`
    int nx, ny, nz;
    Layout lay;               // storage order of the nodes (row or brick layout)
    int tiles_x, tiles_y;     // tile grid in x and y (row layout; one plane per tile row)
    int n_tiles;              // row layout: tiles_x * tiles_y * nz; brick layout: the
                              // bricks holding fluid / 4, rounded up
    int tiles_per_xcd;        // ceil(n_tiles / 8)
    int tx_log2;              // tile width = 1 << tx_log2, height = 256 >> tx_log2
    int pair;                 // FP16 even step with two nodes per lane (k_collide_pair_even)
    int n_segs;               // its 128-node row segments (nx ny nz / 128; a tile is four)
    int row_log2;             // log2(rows per 4096-node block) when whole rows tile the
                              // blocks and a tile is at least a wave wide, else -1
    int uniform_tag;          // model tag of every node (untagged variants)
    int has_force;
    int has_mlp;              // closure parameters uploaded
    double rho0;
    double tau;               // tau (BGK) = tau_plus (TRT)
    double omega;             // 1 / tau
    double omega_minus;       // TRT: 1 / (1/2 + Lambda / (tau - 1/2))
    double smag_c;            // 18 sqrt(2) Cs^2 (implicit Smagorinsky)
    double nu0;               // (tau - 1/2) / 3
    double force[3];
    double bc_u[3];           // velocity imposed on velocity-boundary nodes
    double bc_rho[2];         // density imposed on pressure-boundary nodes (x = 0, x = nx-1)
    MlpDev mlp;
};

// Parameters of the off-step helpers (initialisation, gathers, scatters).
struct AuxParams {
    void *pops;
    const uint8_t *tags;
    int nx, ny, nz;
    Layout lay;               // storage order of tags and populations
    int parity;               // layout parity of the state (0: natural)
    int shifted;              // gathers/scatters of h_i = f_i - w_i rho0 (not f_i)
    double rho0;
    double force[3];
    long long cell0;          // first node of the chunk (range modes)
    long long count;          // nodes in the chunk / in the list
    const long long *cells;   // node list (list mode) or null
    const double *in_rho;     // init: nullable
    const double *in_u;       // init: nullable, 3 planes of `count`
    const double *in_f;       // scatter: Q planes of `count`
    double *out;              // gather output
};

enum GatherMode : int { G_POPS = 0, G_FIELDS = 1, G_CELLS = 2 };

template <int Q, int P>
hipError_t launch_step(const StepParams &p, int ms, bool tagged, int mode, int parity, hipStream_t s);
template <int Q>
// sector_log2: log2 of the nodes per 64-byte storage sector in the lattice's
// precision; odd_fill: also mark the odd-step filler targets.
hipError_t launch_build_mask(const uint8_t *tags, int nx, int ny, int nz, Layout lay, int sector_log2,
                             int odd_fill, uint32_t *mask, hipStream_t s);
template <int Q, int P>
hipError_t launch_init(const AuxParams &a, hipStream_t s);
template <int Q, int P>
hipError_t launch_gather(const AuxParams &a, int gmode, hipStream_t s);
template <int Q, int P>
hipError_t launch_scatter(const AuxParams &a, hipStream_t s);
// Copy the slots that cross a z face between the lattice and buf (see
// lbm_face_pack): face 0 = plane 0, directions with c_z = +1; face 1 =
// plane nz-1, directions with c_z = -1; unpack = 1 copies buf into the lattice.
template <int Q, int P>
hipError_t launch_face(const AuxParams &a, int face, int unpack, void *buf, hipStream_t s);

// Deterministic two-stage sum of the per-tile partials into out[NRED];
// stage1 holds NRED * kFinalizeBlocks doubles.
constexpr int kFinalizeBlocks = 256;
// Classify every wave of every tile of the current tiling (see StepParams::tile_tag).
hipError_t launch_tile_classify(const StepParams &p, int *out, hipStream_t s);

hipError_t launch_finalize(const double *partials, long long partial_stride, int n_tiles, double *stage1, double *out,
                           hipStream_t s);

}  // namespace lbmd
