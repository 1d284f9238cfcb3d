// lbm_probe.hip -- memory-bandwidth probes: plain copy, read-only and
// write-only streams, to measure the HBM ceiling the step kernels are held
// against.  Not part of the method.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "lbm.h"

namespace {

constexpr int kPerLane = 4;  // accesses per lane, issued together

template <typename T>
__device__ __forceinline__ void add_into(uint32_t &acc, const T &v) {
    const uint32_t *w = reinterpret_cast<const uint32_t *>(&v);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) acc += w[k];
}

// Block b moves vectors [b * 1024, (b + 1) * 1024): lane l takes vectors
// l, l + 256, l + 512, l + 768 (each warp-wide access is contiguous).
template <typename T, int KIND>
__global__ __launch_bounds__(256) void k_probe(T *__restrict__ dst, const T *__restrict__ src) {
    const long long base = (long long)blockIdx.x * (256 * kPerLane) + threadIdx.x;
    if constexpr (KIND == 0) {
        T v[kPerLane];
#pragma unroll
        for (int k = 0; k < kPerLane; ++k) v[k] = src[base + k * 256];
#pragma unroll
        for (int k = 0; k < kPerLane; ++k) dst[base + k * 256] = v[k];
    } else if constexpr (KIND == 1) {
        uint32_t acc = 0;
#pragma unroll
        for (int k = 0; k < kPerLane; ++k) add_into(acc, src[base + k * 256]);
        // never true for the probe's inputs in practice; keeps the loads live
        if (acc == 0x9e3779b9u) reinterpret_cast<uint32_t *>(dst)[blockIdx.x] = acc;
    } else {
        T v;
        uint32_t *w = reinterpret_cast<uint32_t *>(&v);
#pragma unroll
        for (int k = 0; k < (int)(sizeof(T) / 4); ++k) w[k] = (uint32_t)threadIdx.x;
#pragma unroll
        for (int k = 0; k < kPerLane; ++k) dst[base + k * 256] = v;
    }
}

template <typename T>
hipError_t launch_probe(int kind, void *dst, const void *src, size_t bytes, hipStream_t s) {
    const size_t blocks = bytes / (sizeof(T) * 256 * kPerLane);
    T *d = static_cast<T *>(dst);
    const T *r = static_cast<const T *>(src);
    if (kind == 0) k_probe<T, 0><<<(unsigned)blocks, 256, 0, s>>>(d, r);
    else if (kind == 1) k_probe<T, 1><<<(unsigned)blocks, 256, 0, s>>>(d, r);
    else k_probe<T, 2><<<(unsigned)blocks, 256, 0, s>>>(d, r);
    return hipGetLastError();
}

}  // namespace

lbm_status lbmd_set_err(lbm_status s, const char *msg);  // lbm_capi.hip

extern "C" lbm_status lbm_probe_bandwidth(int kind, void *dst_dev, const void *src_dev, size_t bytes, int lane_bytes,
                                          void *hip_stream) {
    if (kind < 0 || kind > 2) return lbmd_set_err(LBM_EINVAL, "probe kind must be 0 (copy), 1 (read) or 2 (write)");
    if (lane_bytes != 4 && lane_bytes != 8 && lane_bytes != 16)
        return lbmd_set_err(LBM_EINVAL, "lane_bytes must be 4, 8 or 16");
    if (bytes == 0 || bytes % (4096ull * lane_bytes) != 0)
        return lbmd_set_err(LBM_EINVAL, "bytes must be a positive multiple of 4096 * lane_bytes");
    if (bytes / (4096ull * lane_bytes) > 0x7fffffffull) return lbmd_set_err(LBM_EINVAL, "probe buffer too large");
    if (!dst_dev || (kind != 2 && !src_dev)) return lbmd_set_err(LBM_EINVAL, "null probe buffer");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    hipError_t e;
    if (lane_bytes == 4) e = launch_probe<uint32_t>(kind, dst_dev, src_dev, bytes, s);
    else if (lane_bytes == 8) e = launch_probe<uint2>(kind, dst_dev, src_dev, bytes, s);
    else e = launch_probe<uint4>(kind, dst_dev, src_dev, bytes, s);
    if (e != hipSuccess) return lbmd_set_err(LBM_EHIP, hipGetErrorString(e));
    return LBM_OK;
}
