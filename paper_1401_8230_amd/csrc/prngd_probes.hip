// prngd_probes.hip -- ceilings that bound the PRNGD fill on this GPU:
//   * write probe: coalesced 16-byte stores of n doubles, nothing else
//     (the achievable HBM write bandwidth);
//   * Philox probe: the same Philox4x32-10 blocks a fill of n outputs
//     needs, XOR-folded in registers, one word stored per thread (the
//     integer ALU ceiling of the base generator);
//   * copy probe: n doubles read and written once (the calibration of the
//     HBM byte counters);
//   * Philox+map+store probe: every pair accepted and stored, no
//     compaction and no cross-block scan (the fill without its ordering
//     machinery).
// The probes use the fill's Philox layout but share no control logic
// with it; they exist to price the fill's parts.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/prngd_probe.h"

namespace {

typedef double double2v __attribute__((ext_vector_type(2)));

constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;

struct W4 {
    uint32_t a, b, c, d;
};

__device__ __forceinline__ W4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = uint64_t(kM0) * c0;
        const uint64_t p1 = uint64_t(kM1) * c2;
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(uint32_t(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(uint32_t(p0 >> 32), c3, k1, 0x96);
        c1 = uint32_t(p1);
        c3 = uint32_t(p0);
        c0 = n0;
        c2 = n2;
        k0 += kW0;
        k1 += kW1;
    }
    return {c0, c1, c2, c3};
}

// One 16-byte store per thread over a one-shot grid: workgroups retire in
// dispatch order, so the region being written stays small and moves
// linearly through memory -- the fastest write pattern measured.
__global__ __launch_bounds__(256) void write_probe(double *out, uint64_t n2, double v)
{
    const uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
    const double2v x = {v, v};
    if (i < n2)
        reinterpret_cast<double2v *>(out)[i] = x;
}

__global__ __launch_bounds__(256) void philox_probe(uint32_t *sink, uint64_t blocks, uint64_t seed)
{
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    const uint64_t tid = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
    uint32_t acc = 0;
    for (uint64_t b = tid; b < blocks; b += stride) {
        const W4 r = philox(uint32_t(b), uint32_t(b >> 32), 0u, 7u, uint32_t(seed),
                            uint32_t(seed >> 32));
        acc ^= r.a ^ r.b ^ r.c ^ r.d;
    }
    sink[tid] = acc;
}

// One 16-byte load and one 16-byte store per thread: a plain copy of known
// size, the reference by which HBM byte counters are calibrated.
__global__ __launch_bounds__(256) void copy_probe(double *dst, const double *src, uint64_t n2)
{
    const uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
    if (i < n2)
        reinterpret_cast<double2v *>(dst)[i] = reinterpret_cast<const double2v *>(src)[i];
}

// One Philox block per thread over a one-shot grid, like the write probe.
__global__ __launch_bounds__(256) void philox_store_probe(double *out, uint64_t blocks,
                                                          uint64_t seed, double S)
{
    const uint64_t b = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
    if (b >= blocks)
        return;
    const W4 r = philox(uint32_t(b), uint32_t(b >> 32), 0u, 7u, uint32_t(seed),
                        uint32_t(seed >> 32));
    const double za = __builtin_fma(double(r.a - 1u), 4294967296.0, double(r.b)) * S;
    const double zb = __builtin_fma(double(r.c - 1u), 4294967296.0, double(r.d)) * S;
    const double2v v = {za, zb};
    reinterpret_cast<double2v *>(out)[b] = v;
}

uint32_t grid_for(const void *kernel, uint64_t work)
{
    int dev = 0, cus = 0, nb = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, 256, 0) != hipSuccess)
        return 1024;
    uint64_t g = uint64_t(cus) * uint64_t(nb > 0 ? nb : 1);
    const uint64_t need = (work + 255) / 256;
    if (need < g)
        g = need;
    return uint32_t(g > 0 ? g : 1);
}

}  // namespace

extern "C" {

int prngd_probe_write(double *out, uint64_t n, void *stream)
{
    if (!out || (reinterpret_cast<uintptr_t>(out) & 15u) || (n & 1u))
        return 1;
    const uint64_t n2 = n / 2;
    const uint64_t blocks = (n2 + 255) / 256;
    if (blocks == 0 || blocks > 0xFFFFFFFFull)
        return 1;
    hipLaunchKernelGGL(write_probe, dim3(uint32_t(blocks)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), out, n2, 0.5);
    return hipGetLastError() == hipSuccess ? 0 : 4;
}

int prngd_probe_copy(double *dst, const double *src, uint64_t n, void *stream)
{
    if (!dst || !src || ((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15u) ||
        (n & 1u))
        return 1;
    const uint64_t lo_d = reinterpret_cast<uintptr_t>(dst), lo_s = reinterpret_cast<uintptr_t>(src);
    if (lo_d < lo_s + 8 * n && lo_s < lo_d + 8 * n)
        return 1;                                     // overlapping buffers
    const uint64_t n2 = n / 2;
    const uint64_t blocks = (n2 + 255) / 256;
    if (blocks == 0 || blocks > 0xFFFFFFFFull)
        return 1;
    hipLaunchKernelGGL(copy_probe, dim3(uint32_t(blocks)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), dst, src, n2);
    return hipGetLastError() == hipSuccess ? 0 : 4;
}

int prngd_probe_philox(uint32_t *sink, uint64_t sink_words, uint64_t blocks, void *stream)
{
    if (!sink)
        return 1;
    uint32_t grid = grid_for(reinterpret_cast<const void *>(&philox_probe), blocks);
    if (uint64_t(grid) * 256 > sink_words)
        grid = uint32_t(sink_words / 256);
    if (grid == 0)
        return 1;
    hipLaunchKernelGGL(philox_probe, dim3(grid), dim3(256), 0, static_cast<hipStream_t>(stream),
                       sink, blocks, uint64_t(42));
    return hipGetLastError() == hipSuccess ? 0 : 4;
}

int prngd_probe_philox_store(double *out, uint64_t n, void *stream)
{
    if (!out || (reinterpret_cast<uintptr_t>(out) & 15u) || (n & 1u))
        return 1;
    const uint64_t blocks = n / 2;
    const uint64_t grid = (blocks + 255) / 256;
    if (grid == 0 || grid > 0xFFFFFFFFull)
        return 1;
    hipLaunchKernelGGL(philox_store_probe, dim3(uint32_t(grid)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), out, blocks, uint64_t(42),
                       0x1.0000000200000p-64);
    return hipGetLastError() == hipSuccess ? 0 : 4;
}

}  // extern "C"
