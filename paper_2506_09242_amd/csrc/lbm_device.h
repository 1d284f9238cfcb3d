// lbm_device.h -- device-side lattice tables and compile-time loop helper.
//
// Canonical velocity order (the ABI's): rest; +x,+y,+z; face diagonals
// (1,1,0),(1,-1,0),(1,0,1),(1,0,-1),(0,1,1),(0,1,-1); D3Q27 corners
// (1,1,1),(1,1,-1),(1,-1,1),(1,-1,-1); then the negatives in the same order,
// so the opposite of i in 1..H is i+H (H = (Q-1)/2).  Weights are the
// textbook D3Q19 (1/3, 1/18, 1/36) and D3Q27 (8/27, 2/27, 1/54, 1/216) ones,
// c_s^2 = 1/3.  Every index is a compile-time constant, so the tables fold
// into immediates.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace lbmd {

constexpr int kHalfDirs[13][3] = {
    {1, 0, 0},  {0, 1, 0},  {0, 0, 1},  {1, 1, 0},  {1, -1, 0}, {1, 0, 1},  {1, 0, -1},
    {0, 1, 1},  {0, 1, -1}, {1, 1, 1},  {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};

template <int Q, int I>
struct V {
    static_assert(Q == 19 || Q == 27, "D3Q19 or D3Q27");
    static constexpr int H = (Q - 1) / 2;
    static constexpr int k = I == 0 ? 0 : (I <= H ? I - 1 : I - 1 - H);
    static constexpr int s = I == 0 ? 0 : (I <= H ? 1 : -1);
    static constexpr int x = s * kHalfDirs[k][0];
    static constexpr int y = s * kHalfDirs[k][1];
    static constexpr int z = s * kHalfDirs[k][2];
    static constexpr int opp = I == 0 ? 0 : (I <= H ? I + H : I - H);
    static constexpr int n2 = x * x + y * y + z * z;
    static constexpr double w =
        Q == 19 ? (n2 == 0 ? 1.0 / 3.0 : (n2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0))
                : (n2 == 0 ? 8.0 / 27.0 : (n2 == 1 ? 2.0 / 27.0 : (n2 == 2 ? 1.0 / 54.0 : 1.0 / 216.0)));
};

template <typename F, int... Is>
__device__ __forceinline__ void sfor_impl(F &&f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, Is>{}), ...);
}
// Calls f(integral_constant<int, i>) for i = 0 .. N-1 (fully unrolled).
template <int N, typename F>
__device__ __forceinline__ void sfor(F &&f) {
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

__host__ __device__ inline bool is_fluid_tag(int t) { return t >= 1 && t <= 10; }

// Population layout (blocked structure of arrays).  Node indices are grouped
// in blocks of kBlockNodes consecutive nodes; a block stores its Q slots one
// after another, each slot kBlockNodes contiguous elements, so population i
// of node n is element ((n / B) * Q + i) * B + n % B.  A wave still touches
// contiguous 64-node runs of one slot, and the Q streams a block reads and
// writes lie within Q * B elements of each other instead of a whole lattice
// apart, which the memory serves about 10% faster than plain per-slot planes.
constexpr int kBlockLog2 = 12;
constexpr long long kBlockNodes = 1ll << kBlockLog2;

// Element index of population 0 of the node with storage index n (0 <= n < 2^31).
template <int Q>
__device__ __forceinline__ long long pop_base(int n) {
    const unsigned b = (unsigned)n >> kBlockLog2;
    return (long long)((unsigned long long)b * (unsigned)(Q << kBlockLog2)) + (n & (int)(kBlockNodes - 1));
}
// Storage order of the nodes.  Every per-node array on the device (the
// populations' blocks, tags, neighbour masks) is indexed by a storage index
// s = lay_z(z) + lay_y(y) + lay_x(x), separable in the three coordinates:
//  - row layout (brick == 0): s = (z ny + y) nx + x, the natural order;
//  - brick layout (brick == 1, nx, ny, nz multiples of 16): the lattice is cut
//    into 16^3 blocks (4096 nodes, block index (z/16 * nby + y/16) * nbx +
//    x/16), each block into 64 bricks of 4^3 nodes (brick index
//    (z/4 % 4) 16 + (y/4 % 4) 4 + x/4 % 4) and each brick ordered x fastest;
//    a 64-byte sector of FP32 storage is then a 4 x 4 x 1 patch instead of 16
//    nodes of one row, which a porous medium fills with fluid far more often.
struct Layout {
    int brick, nx, nxy, nbx, nbxy;
    __host__ __device__ int x(int v) const { return brick ? ((v >> 4) << 12) | (((v >> 2) & 3) << 6) | (v & 3) : v; }
    __host__ __device__ int y(int v) const {
        return brick ? (v >> 4) * (nbx << 12) + ((((v >> 2) & 3) << 8) | ((v & 3) << 2)) : v * nx;
    }
    __host__ __device__ int z(int v) const {
        return brick ? (v >> 4) * (nbxy << 12) + ((((v >> 2) & 3) << 10) | ((v & 3) << 4)) : v * nxy;
    }
    __host__ __device__ int at(int vx, int vy, int vz) const { return z(vz) + y(vy) + x(vx); }
};
__host__ __device__ inline Layout make_layout(int brick, int nx, int ny) {
    return Layout{brick, nx, nx * ny, nx >> 4, (nx >> 4) * (ny >> 4)};
}

// Element offset of slot i from population 0 of the same node.
__device__ __forceinline__ constexpr long long slot_off(int i) { return (long long)i << kBlockLog2; }

// Storage / compute types per precision (lbm_prec).
template <int P>
struct Prec;
template <>
struct Prec<0> {
    using S = double;
    using C = double;
};
template <>
struct Prec<1> {
    using S = float;
    using C = float;
};
template <>
struct Prec<2> {
    using S = _Float16;
    using C = float;
};

}  // namespace lbmd
