// lbm_mlp.hip -- learned eddy-viscosity closure: parameter packing, the
// standalone inference kernel (same device code as the fused collision), the
// box filter that turns a fine lattice into training samples, and the FP32
// training kernels (forward, backward, deterministic gradient reduction, Adam).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"
#include "lbm_mlp_device.h"

using namespace lbmd;

lbm_status lbmd_fail_hip(lbm_lattice *lat, hipError_t e, const char *what);
lbm_status lbmd_set_err(lbm_status s, const char *msg);
lbm_config lbmd_config(const lbm_lattice *lat);
hipStream_t lbmd_stream(const lbm_lattice *lat);
bool lbmd_failed(const lbm_lattice *lat);
void lbmd_set_mlp(lbm_lattice *lat, void *block, const MlpDev &m);
void *lbmd_mlp_block(lbm_lattice *lat);
void lbmd_clear_mlp(lbm_lattice *lat);
lbm_status lbmd_fields_device(lbm_lattice *lat, double *d_out);

#define HIPCHK(lat, expr)                                              \
    do {                                                               \
        hipError_t e_ = (expr);                                        \
        if (e_ != hipSuccess) return lbmd_fail_hip((lat), e_, #expr);  \
    } while (0)

namespace {

// Offsets in the packed FP32 parameter vector (see lbm.h).
constexpr int OW1 = 0, OB1 = 224, OW2 = 256, OB2 = 1280, OW3 = 1312, OB3 = 1344, OMEAN = 1345, OSTD = 1352;
constexpr int NP = LBM_MLP_NPARAMS;   // 1359
constexpr int NTRAIN = 1345;          // trainable entries (weights and biases)

// FP32 -> BF16 bit pattern, round to nearest even (NaN kept quiet).
uint16_t bf16_bits(float v) {
    uint32_t b;
    std::memcpy(&b, &v, 4);
    if ((b & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((b >> 16) | 0x40u);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

// Device block (see MlpDev): w1p[32][8] u16 | w2p[2][2][32][8] u16 | w3p[2][16] u16 |
// b1p[2][16] b2p[2][16] b3[1] pad[3] mean[7] pad inv_sd[7] pad (floats).  "Accumulator
// order" of lane group g: entry r is neuron 8 (r / 4) + 4 g + r % 4 (lbm_mlp_device.h).
constexpr size_t kW3Off = (256 + 1024) * 2, kFloatOff = kW3Off + 32 * 2;
constexpr size_t kBlockBytes = kFloatOff + (32 + 32 + 4 + 8 + 8) * 4;

int acc_neuron(int r, int g) { return 8 * (r / 4) + 4 * g + (r % 4); }

void pack_block(const float *P, std::vector<unsigned char> &out) {
    out.assign(kBlockBytes, 0);
    uint16_t *w1p = reinterpret_cast<uint16_t *>(out.data());
    uint16_t *w2p = w1p + 256;
    uint16_t *w3p = reinterpret_cast<uint16_t *>(out.data() + kW3Off);
    float *fl = reinterpret_cast<float *>(out.data() + kFloatOff);
    for (int o = 0; o < 32; ++o)
        for (int s = 0; s < 8; ++s) w1p[o * 8 + s] = s < 7 ? bf16_bits(P[OW1 + o * 7 + s]) : 0;
    // W2 as the A operands of the two layer-2 products: product p, lane group g,
    // row i, K slot s holds W2[i][neuron], the neuron that accumulator register
    // 8p + s of lane group g holds after layer 1
    for (int pr = 0; pr < 2; ++pr)
        for (int g = 0; g < 2; ++g)
            for (int i = 0; i < 32; ++i)
                for (int s = 0; s < 8; ++s)
                    w2p[((pr * 2 + g) * 32 + i) * 8 + s] = bf16_bits(P[OW2 + i * 32 + acc_neuron(8 * pr + s, g)]);
    for (int g = 0; g < 2; ++g)
        for (int r = 0; r < 16; ++r) {
            const int o = acc_neuron(r, g);
            w3p[g * 16 + r] = bf16_bits(P[OW3 + o]);
            fl[g * 16 + r] = P[OB1 + o];
            fl[32 + g * 16 + r] = P[OB2 + o];
        }
    fl[64] = P[OB3];
    for (int k = 0; k < 7; ++k) {
        fl[68 + k] = P[OMEAN + k];
        fl[76 + k] = 1.0f / P[OSTD + k];
    }
}

MlpDev block_view(void *d) {
    MlpDev m;
    unsigned char *b = static_cast<unsigned char *>(d);
    float *fl = reinterpret_cast<float *>(b + kFloatOff);
    m.w1 = reinterpret_cast<uint16_t *>(b);
    m.w2 = m.w1 + 256;
    m.w3 = reinterpret_cast<uint16_t *>(b + kW3Off);
    m.b1 = fl;
    m.b2 = fl + 32;
    m.b3 = fl + 64;
    m.mean = fl + 68;
    m.inv_sd = fl + 76;
    return m;
}

lbm_status check_params(const float *P) {
    for (int k = 0; k < NP; ++k)
        if (!std::isfinite(P[k])) return lbmd_set_err(LBM_EINVAL, "closure parameters must be finite");
    for (int k = 0; k < 7; ++k)
        if (!(P[OSTD + k] > 0.0f)) return lbmd_set_err(LBM_EINVAL, "closure std entries must be > 0");
    return LBM_OK;
}

}  // namespace

void lbmd_free_mlp(lbm_lattice *lat) {
    void *b = lbmd_mlp_block(lat);
    if (b) (void)hipFree(b);
    lbmd_clear_mlp(lat);
}

extern "C" lbm_status lbm_set_mlp(lbm_lattice *lat, const float *params_host, size_t n) {
    if (!lat) return lbmd_set_err(LBM_EINVAL, "null lattice handle");
    if (lbmd_failed(lat)) return lbmd_set_err(LBM_ESTATE, "lattice handle failed earlier");
    if (!params_host || n != (size_t)NP) return lbmd_set_err(LBM_EINVAL, "expected LBM_MLP_NPARAMS floats");
    lbm_status s = check_params(params_host);
    if (s != LBM_OK) return s;
    std::vector<unsigned char> blk;
    pack_block(params_host, blk);
    void *d = lbmd_mlp_block(lat);
    if (!d) HIPCHK(lat, hipMalloc(&d, kBlockBytes));
    hipStream_t st = lbmd_stream(lat);
    hipError_t e = hipMemcpyAsync(d, blk.data(), kBlockBytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipFree(d);
        lbmd_clear_mlp(lat);
        return lbmd_fail_hip(lat, e, "closure upload");
    }
    lbmd_set_mlp(lat, d, block_view(d));
    return LBM_OK;
}

// ------------------------------------------------------------ inference
namespace lbmd {
__global__ __launch_bounds__(256) void k_mlp_infer(MlpDev m, float nu0, const float *feat, long long n,
                                                   float *nut) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    float x[7];
#pragma unroll
    for (int k = 0; k < 7; ++k) x[k] = t < n ? feat[t * 7 + k] : m.mean[k];
    const float sp = mlp_wave_eval(m, x);  // every lane takes part
    if (t < n) nut[t] = nu0 * sp;
}
}  // namespace lbmd

extern "C" lbm_status lbm_mlp_infer(const float *params_host, double nu0, const float *feat_dev, int64_t n,
                                    float *nut_dev, void *hip_stream) {
    if (!params_host || (n > 0 && (!feat_dev || !nut_dev)) || n < 0)
        return lbmd_set_err(LBM_EINVAL, "bad arguments to lbm_mlp_infer");
    lbm_status s = check_params(params_host);
    if (s != LBM_OK) return s;
    if (n == 0) return LBM_OK;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    std::vector<unsigned char> blk;
    pack_block(params_host, blk);
    void *d = nullptr;
    HIPCHK(nullptr, hipMalloc(&d, kBlockBytes));
    hipError_t e = hipMemcpyAsync(d, blk.data(), kBlockBytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        k_mlp_infer<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(block_view(d), (float)nu0, feat_dev, n, nut_dev);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    if (e != hipSuccess) return lbmd_fail_hip(nullptr, e, "lbm_mlp_infer");
    return LBM_OK;
}

// ------------------------------------------------------------ box filter
namespace lbmd {
// fields: FP64 planes rho, ux, uy, uz of the fine lattice.  coarse: FP64
// planes rho_bar, U (3), T (6: xx yy zz xy xz yz) per coarse node.
__global__ __launch_bounds__(256) void k_box_filter(const double *fields, long long nfine, int nx, int ny, int fct,
                                                    int cx, int cy, int cz, double *coarse) {
    const long long nc = (long long)cx * cy * cz;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= nc) return;
    const int X = (int)(t % cx), Y = (int)((t / cx) % cy), Z = (int)(t / ((long long)cx * cy));
    double sr = 0, sx = 0, sy = 0, sz = 0, txx = 0, tyy = 0, tzz = 0, txy = 0, txz = 0, tyz = 0;
    for (int dz = 0; dz < fct; ++dz)
        for (int dy = 0; dy < fct; ++dy)
            for (int dx = 0; dx < fct; ++dx) {
                const long long n = ((long long)(Z * fct + dz) * ny + (Y * fct + dy)) * nx + (X * fct + dx);
                const double r = fields[n], ux = fields[nfine + n], uy = fields[2 * nfine + n],
                             uz = fields[3 * nfine + n];
                sr += r;
                sx += r * ux;
                sy += r * uy;
                sz += r * uz;
                txx += r * ux * ux;
                tyy += r * uy * uy;
                tzz += r * uz * uz;
                txy += r * ux * uy;
                txz += r * ux * uz;
                tyz += r * uy * uz;
            }
    const double vol = (double)fct * fct * fct;
    const double Ux = sx / sr, Uy = sy / sr, Uz = sz / sr;
    coarse[t] = sr / vol;
    coarse[nc + t] = Ux;
    coarse[2 * nc + t] = Uy;
    coarse[3 * nc + t] = Uz;
    coarse[4 * nc + t] = txx / sr - Ux * Ux;
    coarse[5 * nc + t] = tyy / sr - Uy * Uy;
    coarse[6 * nc + t] = tzz / sr - Uz * Uz;
    coarse[7 * nc + t] = txy / sr - Ux * Uy;
    coarse[8 * nc + t] = txz / sr - Ux * Uz;
    coarse[9 * nc + t] = tyz / sr - Uy * Uz;
}

__global__ __launch_bounds__(256) void k_closure_targets(const double *coarse, int cx, int cy, int cz, double nu_c,
                                                         float *feat, float *target) {
    const long long nc = (long long)cx * cy * cz;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= nc) return;
    const int X = (int)(t % cx), Y = (int)((t / cx) % cy), Z = (int)(t / ((long long)cx * cy));
    auto at = [&](int comp, int x, int y, int z) {
        x = (x + cx) % cx;
        y = (y + cy) % cy;
        z = (z + cz) % cz;
        return coarse[comp * nc + ((long long)z * cy + y) * cx + x];
    };
    // G[a][b] = dU_b / dx_a, second-order central differences.
    double G[3][3];
    for (int b = 0; b < 3; ++b) {
        G[0][b] = 0.5 * (at(1 + b, X + 1, Y, Z) - at(1 + b, X - 1, Y, Z));
        G[1][b] = 0.5 * (at(1 + b, X, Y + 1, Z) - at(1 + b, X, Y - 1, Z));
        G[2][b] = 0.5 * (at(1 + b, X, Y, Z + 1) - at(1 + b, X, Y, Z - 1));
    }
    double S[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) S[a][b] = 0.5 * (G[a][b] + G[b][a]);
    const double T[3][3] = {{coarse[4 * nc + t], coarse[7 * nc + t], coarse[8 * nc + t]},
                            {coarse[7 * nc + t], coarse[5 * nc + t], coarse[9 * nc + t]},
                            {coarse[8 * nc + t], coarse[9 * nc + t], coarse[6 * nc + t]}};
    const double tr = (T[0][0] + T[1][1] + T[2][2]) / 3.0;
    double num = 0.0, ss = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            num += (T[a][b] - (a == b ? tr : 0.0)) * S[a][b];
            ss += S[a][b] * S[a][b];
        }
    const double nut = fmax(0.0, -num / (2.0 * ss + 1e-30));
    const double rho = coarse[t];
    const double tau_e = 3.0 * (nu_c + nut) + 0.5;
    const double c = -(2.0 / 3.0) * rho * tau_e;
    feat[t * 7 + 0] = (float)(c * S[0][0]);
    feat[t * 7 + 1] = (float)(c * S[1][1]);
    feat[t * 7 + 2] = (float)(c * S[2][2]);
    feat[t * 7 + 3] = (float)(c * S[0][1]);
    feat[t * 7 + 4] = (float)(c * S[0][2]);
    feat[t * 7 + 5] = (float)(c * S[1][2]);
    feat[t * 7 + 6] = (float)rho;
    target[t] = (float)(nut / nu_c);
}
}  // namespace lbmd

extern "C" lbm_status lbm_filter_snapshot(lbm_lattice *fine, int factor, float *feat_dev, float *target_dev) {
    if (!fine) return lbmd_set_err(LBM_EINVAL, "null lattice handle");
    if (lbmd_failed(fine)) return lbmd_set_err(LBM_ESTATE, "lattice handle failed earlier");
    const lbm_config c = lbmd_config(fine);
    if (factor < 1 || c.nx % factor || c.ny % factor || c.nz % factor)
        return lbmd_set_err(LBM_EINVAL, "lattice sizes must be divisible by the filter factor");
    if (!feat_dev || !target_dev) return lbmd_set_err(LBM_EINVAL, "null output");
    const long long N = (long long)c.nx * c.ny * c.nz;
    const int cx = c.nx / factor, cy = c.ny / factor, cz = c.nz / factor;
    const long long nc = (long long)cx * cy * cz;
    hipStream_t st = lbmd_stream(fine);
    double *d_fields = nullptr, *d_coarse = nullptr;
    HIPCHK(fine, hipMalloc(&d_fields, (size_t)N * 4 * sizeof(double)));
    hipError_t e = hipMalloc(&d_coarse, (size_t)nc * 10 * sizeof(double));
    if (e != hipSuccess) {
        (void)hipFree(d_fields);
        return lbmd_fail_hip(fine, e, "hipMalloc coarse");
    }
    lbm_status s = lbmd_fields_device(fine, d_fields);
    if (s == LBM_OK) {
        const unsigned blocks = (unsigned)((nc + 255) / 256);
        k_box_filter<<<blocks, 256, 0, st>>>(d_fields, N, c.nx, c.ny, factor, cx, cy, cz, d_coarse);
        const double nu_c = (c.tau - 0.5) / 3.0 / factor;
        k_closure_targets<<<blocks, 256, 0, st>>>(d_coarse, cx, cy, cz, nu_c, feat_dev, target_dev);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) s = lbmd_fail_hip(fine, e, "closure filter");
    }
    (void)hipFree(d_fields);
    (void)hipFree(d_coarse);
    return s;
}

// ------------------------------------------------------------ training
namespace lbmd {
constexpr int ACT = 136;  // per-sample record: xhat 7 | h1 32 | h2 32 | d1 32 | d2 32 | d3 1
constexpr int A_X = 0, A_H1 = 7, A_H2 = 39, A_D1 = 71, A_D2 = 103, A_D3 = 135;

// Forward and backward of one sample per thread (FP32); loss = scale * (y - t)^2.
__global__ __launch_bounds__(256) void k_fwd_bwd(const float *P, const float *feat, const float *target,
                                                 const long long *idx, long long base, int nb, long long n,
                                                 float scale, float *act, float *loss) {
    __shared__ float sp[NP];
    for (int k = threadIdx.x; k < NP; k += 256) sp[k] = P[k];
    __syncthreads();
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= nb) return;
    long long s = idx ? idx[base + b] : base + b;
    float *r = act + (long long)b * ACT;
    if (s < 0 || s >= n) {  // out-of-range sample index: contributes nothing
        for (int k = 0; k < ACT; ++k) r[k] = 0.0f;
        loss[b] = 0.0f;
        return;
    }
    float x[7];
    for (int k = 0; k < 7; ++k) {
        x[k] = (feat[s * 7 + k] - sp[OMEAN + k]) / sp[OSTD + k];
        r[A_X + k] = x[k];
    }
    float z1[32], h1[32], z2[32], h2[32];
    for (int o = 0; o < 32; ++o) {
        float a = sp[OB1 + o];
        for (int k = 0; k < 7; ++k) a += sp[OW1 + o * 7 + k] * x[k];
        z1[o] = a;
        h1[o] = a > 0.0f ? a : 0.0f;
        r[A_H1 + o] = h1[o];
    }
    for (int o = 0; o < 32; ++o) {
        float a = sp[OB2 + o];
        for (int k = 0; k < 32; ++k) a += sp[OW2 + o * 32 + k] * h1[k];
        z2[o] = a;
        h2[o] = a > 0.0f ? a : 0.0f;
        r[A_H2 + o] = h2[o];
    }
    float z3 = sp[OB3];
    for (int k = 0; k < 32; ++k) z3 += sp[OW3 + k] * h2[k];
    const float y = softplus_f(z3);
    const float res = y - target[s];
    loss[b] = scale * res * res;
    const float sig = 1.0f / (1.0f + expf(-z3));
    const float d3 = scale * 2.0f * res * sig;
    r[A_D3] = d3;
    float d2[32];
    for (int o = 0; o < 32; ++o) {
        d2[o] = z2[o] > 0.0f ? d3 * sp[OW3 + o] : 0.0f;
        r[A_D2 + o] = d2[o];
    }
    for (int k = 0; k < 32; ++k) {
        float a = 0.0f;
        for (int o = 0; o < 32; ++o) a += sp[OW2 + o * 32 + k] * d2[o];
        r[A_D1 + k] = z1[k] > 0.0f ? a : 0.0f;
    }
}

// Partial gradients of `chunk` consecutive samples; part[c][k], k < NP, and
// part[c][NP] = partial loss.  Fixed summation order.
__global__ __launch_bounds__(256) void k_grad_partial(const float *act, const float *loss, int nb, int chunk,
                                                      float *part) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (k > NP) return;
    const int b0 = c * chunk, b1 = min(nb, b0 + chunk);
    float g = 0.0f;
    if (k == NP) {
        for (int b = b0; b < b1; ++b) g += loss[b];
    } else if (k < OB1) {
        const int o = k / 7, i = k % 7;
        for (int b = b0; b < b1; ++b) g += act[(long long)b * ACT + A_D1 + o] * act[(long long)b * ACT + A_X + i];
    } else if (k < OW2) {
        const int o = k - OB1;
        for (int b = b0; b < b1; ++b) g += act[(long long)b * ACT + A_D1 + o];
    } else if (k < OB2) {
        const int o = (k - OW2) / 32, i = (k - OW2) % 32;
        for (int b = b0; b < b1; ++b) g += act[(long long)b * ACT + A_D2 + o] * act[(long long)b * ACT + A_H1 + i];
    } else if (k < OW3) {
        const int o = k - OB2;
        for (int b = b0; b < b1; ++b) g += act[(long long)b * ACT + A_D2 + o];
    } else if (k < OB3) {
        const int i = k - OW3;
        for (int b = b0; b < b1; ++b) g += act[(long long)b * ACT + A_D3] * act[(long long)b * ACT + A_H2 + i];
    } else if (k == OB3) {
        for (int b = b0; b < b1; ++b) g += act[(long long)b * ACT + A_D3];
    }
    part[(long long)c * (NP + 1) + k] = g;
}

// Plain zero fill (used instead of memset so callers may capture the work).
__global__ __launch_bounds__(256) void k_zero(float *p, long long n) {
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t < n) p[t] = 0.0f;
}

// Sum chunk partials in order: out[k] = sum_c part[c][k], k <= NP.
__global__ __launch_bounds__(256) void k_grad_sum(const float *part, int nchunks, float *out) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k > NP) return;
    float g = 0.0f;
    for (int c = 0; c < nchunks; ++c) g += part[(long long)c * (NP + 1) + k];
    out[k] = g;
}

// One Adam step from the chunk partials; loss_log[epoch] += batch loss * w.
__global__ __launch_bounds__(256) void k_adam(const float *part, int nchunks, float *P, float *m, float *v, float lr,
                                              float bc1, float bc2, float *loss_log, int epoch, float w) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k > NP) return;
    float g = 0.0f;
    for (int c = 0; c < nchunks; ++c) g += part[(long long)c * (NP + 1) + k];
    if (k == NP) {
        loss_log[epoch] += g * w;
        return;
    }
    if (k >= NTRAIN) return;
    const float mk = 0.9f * m[k] + 0.1f * g;
    const float vk = 0.999f * v[k] + 0.001f * g * g;
    m[k] = mk;
    v[k] = vk;
    P[k] -= lr * (mk / bc1) / (sqrtf(vk / bc2) + 1e-8f);
}
}  // namespace lbmd

namespace {
struct TrainScratch {
    float *act = nullptr, *loss = nullptr, *part = nullptr, *m = nullptr, *v = nullptr;
    ~TrainScratch() {
        for (float *p : {act, loss, part, m, v})
            if (p) (void)hipFree(p);
    }
};
}  // namespace

extern "C" lbm_status lbm_mlp_grad(const float *params_dev, const float *feat_dev, const float *target_dev, int64_t n,
                                   float *grad_dev, float *loss_dev, void *hip_stream) {
    if (!params_dev || !feat_dev || !target_dev || !grad_dev || !loss_dev || n < 1)
        return lbmd_set_err(LBM_EINVAL, "bad arguments to lbm_mlp_grad");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    constexpr int SUB = 65536, CHUNK = 1024;
    const long long nsub = (n + SUB - 1) / SUB;
    const long long nchunks = nsub * (SUB / CHUNK);
    TrainScratch sc;
    HIPCHK(nullptr, hipMalloc(&sc.act, (size_t)SUB * ACT * sizeof(float)));
    HIPCHK(nullptr, hipMalloc(&sc.loss, (size_t)SUB * sizeof(float)));
    HIPCHK(nullptr, hipMalloc(&sc.part, (size_t)nchunks * (NP + 1) * sizeof(float)));
    const long long npart = nchunks * (NP + 1);
    k_zero<<<(unsigned)((npart + 255) / 256), 256, 0, st>>>(sc.part, npart);
    const float scale = 1.0f / (float)n;
    for (long long sb = 0; sb < nsub; ++sb) {
        const long long base = sb * SUB;
        const int nb = (int)std::min<long long>(SUB, n - base);
        k_fwd_bwd<<<(nb + 255) / 256, 256, 0, st>>>(params_dev, feat_dev, target_dev, nullptr, base, nb, n,
                                                   scale, sc.act, sc.loss);
        const dim3 g((NP + 1 + 255) / 256, (nb + CHUNK - 1) / CHUNK);
        k_grad_partial<<<g, 256, 0, st>>>(sc.act, sc.loss, nb, CHUNK, sc.part + sb * (SUB / CHUNK) * (NP + 1));
    }
    k_grad_sum<<<(NP + 1 + 255) / 256, 256, 0, st>>>(sc.part, (int)nchunks, sc.act);
    HIPCHK(nullptr, hipGetLastError());
    HIPCHK(nullptr, hipMemcpyAsync(grad_dev, sc.act, NP * sizeof(float), hipMemcpyDeviceToDevice, st));
    HIPCHK(nullptr, hipMemcpyAsync(loss_dev, sc.act + NP, sizeof(float), hipMemcpyDeviceToDevice, st));
    HIPCHK(nullptr, hipStreamSynchronize(st));
    return LBM_OK;
}

extern "C" lbm_status lbm_mlp_train(float *params_dev, const float *feat_dev, const float *target_dev, int64_t n,
                                    const int64_t *perm_dev, int batch, int epochs, double lr, float *loss_log_dev,
                                    void *hip_stream) {
    if (!params_dev || !feat_dev || !target_dev || !perm_dev || !loss_log_dev || n < 1 || batch < 1 ||
        batch > 65536 || epochs < 0 || !(lr > 0.0))
        return lbmd_set_err(LBM_EINVAL, "bad arguments to lbm_mlp_train");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    constexpr int CHUNK = 256;
    const int maxchunks = (batch + CHUNK - 1) / CHUNK;
    TrainScratch sc;
    HIPCHK(nullptr, hipMalloc(&sc.act, (size_t)batch * ACT * sizeof(float)));
    HIPCHK(nullptr, hipMalloc(&sc.loss, (size_t)batch * sizeof(float)));
    HIPCHK(nullptr, hipMalloc(&sc.part, (size_t)maxchunks * (NP + 1) * sizeof(float)));
    HIPCHK(nullptr, hipMalloc(&sc.m, NP * sizeof(float)));
    HIPCHK(nullptr, hipMalloc(&sc.v, NP * sizeof(float)));
    k_zero<<<(NP + 255) / 256, 256, 0, st>>>(sc.m, NP);
    k_zero<<<(NP + 255) / 256, 256, 0, st>>>(sc.v, NP);
    k_zero<<<(unsigned)((epochs + 255) / 256 + 1), 256, 0, st>>>(loss_log_dev, epochs);
    const long long nbatches = (n + batch - 1) / batch;
    long long step = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        for (long long bi = 0; bi < nbatches; ++bi) {
            const long long base = bi * batch;
            const int nb = (int)std::min<long long>(batch, n - base);
            const int nch = (nb + CHUNK - 1) / CHUNK;
            k_fwd_bwd<<<(nb + 255) / 256, 256, 0, st>>>(params_dev, feat_dev, target_dev,
                                                       reinterpret_cast<const long long *>(perm_dev),
                                                       (long long)ep * n + base, nb, n, 1.0f / nb, sc.act,
                                                       sc.loss);
            const dim3 g((NP + 1 + 255) / 256, nch);
            k_grad_partial<<<g, 256, 0, st>>>(sc.act, sc.loss, nb, CHUNK, sc.part);
            ++step;
            const float bc1 = 1.0f - std::pow(0.9f, (float)step);
            const float bc2 = 1.0f - std::pow(0.999f, (float)step);
            k_adam<<<(NP + 1 + 255) / 256, 256, 0, st>>>(sc.part, nch, params_dev, sc.m, sc.v, (float)lr, bc1, bc2,
                                                        loss_log_dev, ep, 1.0f / (float)nbatches);
        }
        HIPCHK(nullptr, hipGetLastError());
    }
    HIPCHK(nullptr, hipStreamSynchronize(st));
    return LBM_OK;
}
