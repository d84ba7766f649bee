// prngd_k_misc.hip -- small kernels of the runtime (plan parity, position
// writes, clearing, tile maps), the kernel lookup by family and launch
// shape, and the launch wrappers.
#include <type_traits>

#include "prngd_device.hpp"

namespace prngd {
namespace {

// The two-level scan of the counted single fill.
// Level 1: workgroup b scans the counts of chunks [b B, (b + 1) B)
// (B = kScanBlock, 4 per thread), writes each chunk's offset in its block
// and the block's total to block_offs[b].
__global__ __launch_bounds__(1024) void counted_scan_blocks_kernel(LaunchArgs args)
{
    __shared__ uint32_t s_wave[16];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint32_t total = args.total_tiles;
    const uint64_t c0 = uint64_t(blockIdx.x) * kScanBlock + 4u * tid;
    uint32_t v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
        v[i] = c0 + uint32_t(i) < total ? args.chunk_counts[c0 + i] : 0u;
    const uint32_t mine = v[0] + v[1] + v[2] + v[3];
    const uint32_t incl = wave_incl_scan(mine, lane);
    if (lane == 63)
        s_wave[wave] = incl;
    __syncthreads();
    uint32_t before = 0, sum = 0;
#pragma unroll
    for (uint32_t w = 0; w < 16; ++w) {
        const uint32_t t = s_wave[w];
        before += w < wave ? t : 0u;
        sum += t;
    }
    uint32_t run = before + incl - mine;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (c0 + uint32_t(i) < total)
            args.chunk_offs[c0 + i] = run;
        run += v[i];
    }
    if (tid == 0)
        args.block_offs[blockIdx.x] = sum;
}

// Level 2: one workgroup turns the block totals (at most kScanBlocksMax)
// into exclusive offsets, in place.
__global__ __launch_bounds__(1024) void counted_scan_top_kernel(LaunchArgs args)
{
    __shared__ uint64_t s_wave[16];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint32_t nblocks = (args.total_tiles + kScanBlock - 1) / kScanBlock;
    const uint64_t mine = tid < nblocks ? args.block_offs[tid] : 0u;
    uint64_t incl = mine;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t u = uint64_t(uint32_t(__shfl_up(uint32_t(incl), d, 64))) |
                           uint64_t(uint32_t(__shfl_up(uint32_t(incl >> 32), d, 64))) << 32;
        if (lane >= uint32_t(d))
            incl += u;
    }
    if (lane == 63)
        s_wave[wave] = incl;
    __syncthreads();
    uint64_t before = 0;
    for (uint32_t w = 0; w < wave; ++w)
        before += s_wave[w];
    if (tid < nblocks)
        args.block_offs[tid] = before + incl - mine;
}

// Toggles a resident plan's replay parity after all of a replay's fills.
__global__ void toggle_flip_kernel(uint32_t *flip)
{
    *flip ^= 1u;
}

// Sets a handle's position slot (both halves, so either parity reads it).
__global__ void set_counter_kernel(uint64_t *slot, uint64_t value)
{
    slot[0] = value;
    slot[1] = value;
}

// RANMAR states: both slots of handle state `dst` (and, if `slot` is not
// null, both pair counters) set from words [0, kRanmarRow) of one record.
__global__ void ranmar_set_states_kernel(const RanmarInit *inits, uint32_t count)
{
    const RanmarInit &r = inits[blockIdx.x];
    for (uint32_t i = threadIdx.x; i < kRanmarRow; i += blockDim.x) {
        r.dst->slot[0][i] = r.words[i];
        r.dst->slot[1][i] = r.words[i];
    }
    if (threadIdx.x == 0 && r.slot) {
        r.slot[0] = r.counter;
        r.slot[1] = r.counter;
    }
}

__global__ void ranmar_set_state_kernel(RanmarInit r)
{
    for (uint32_t i = threadIdx.x; i < kRanmarRow; i += blockDim.x) {
        r.dst->slot[0][i] = r.words[i];
        r.dst->slot[1][i] = r.words[i];
    }
    if (threadIdx.x == 0 && r.slot) {
        r.slot[0] = r.counter;
        r.slot[1] = r.counter;
    }
}

__global__ void zero_words_kernel(uint64_t *p, size_t n)
{
    for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
         i += size_t(gridDim.x) * blockDim.x)
        p[i] = 0;
}

// tile_seg[tile_begin .. tile_begin + ntiles) = segment index, one
// workgroup per segment.
__global__ void expand_tiles_kernel(const Segment *segs, uint32_t nseg, uint32_t *tile_seg)
{
    for (uint32_t s = blockIdx.x; s < nseg; s += gridDim.x) {
        const uint32_t b = segs[s].tile_begin, c = segs[s].ntiles;
        for (uint32_t i = threadIdx.x; i < c; i += blockDim.x)
            tile_seg[b + i] = s;
    }
}
// The chunk-speculative batch fill's prologue: one thread per segment
// writes the segment's record for this launch (start chunk and offset,
// output, the position slot half it writes, the chunk bounds).
__global__ void chunk_prep_kernel(LaunchArgs args)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= args.nseg)
        return;
    const Segment s = args.segs[i];
    const uint32_t par = (s.parity ^ read_flip(args)) & 1u;
    const uint64_t c0 = s.counter[par];
    const uint32_t sh = args.chunk_shift;
    const uint64_t P = uint64_t(1) << sh;
    ChunkSeg r;
    r.seed = s.seed;
    r.out = s.out;
    r.w0 = c0 >> sh;
    r.n = s.n;
    r.next_counter = s.counter + (par ^ 1u);
    r.stream_id = s.stream_id;
    r.lo0 = uint32_t(c0 & (P - 1));
    r.tile_begin = s.tile_begin;
    r.ntiles = s.ntiles;
    // n < 2^38: both fit in 32 bits
    r.k_full = uint32_t((s.n + r.lo0 - 1) >> sh);
    r.k_end = uint32_t((s.n + r.lo0 + (P - 1)) >> sh);
    args.chunk_segs[i] = r;
}

}  // namespace

// The routers below take a family with or without FAM_ANY_MAP and pick
// the kernels built for it.
template <class F>
static const void *by_map(uint32_t fam, F &&f)
{
    return (fam & FAM_ANY_MAP) ? f(std::integral_constant<uint32_t, FAM_ANY_MAP>())
                               : f(std::integral_constant<uint32_t, 0u>());
}

// The speculative fill kernel (single-segment or batched form) or its
// repair kernel for (family, threads per workgroup, pairs per lane); null
// for shapes without one.
const void *spec_kernel_for(uint32_t fam, uint32_t threads, uint32_t ppl, bool repair,
                            bool single, bool hold)
{
    if (fam_base(fam) == FAM_MRG || fam_base(fam) == FAM_MIXED) {
        // the MRG fill always holds its window before storing
        if (threads != kMrgBlockThreads || (!hold && !repair))
            return nullptr;
        return by_map(fam, [&](auto m) {
            return mrg_spec_kernel_for<decltype(m)::value>(fam, ppl, repair, single);
        });
    }
    return by_map(fam, [&](auto m) {
        return philox_spec_kernel_for<decltype(m)::value>(fam, threads, ppl, repair, single, hold);
    });
}

// The kernel for (family, threads per workgroup, pairs per lane), either
// the look-back kernel or the segment-sequential one (seq), or null if
// that shape is not instantiated.
const void *fill_kernel_for(uint32_t fam, uint32_t threads, uint32_t ppl, bool seq)
{
    const uint32_t b = fam_base(fam);
    if (b == FAM_PHILOX || b == FAM_ENUM || b == FAM_PHILOX32)
        return by_map(fam, [&](auto m) {
            return philox_fill_kernel_for<decltype(m)::value>(fam, threads, ppl, seq);
        });
    if (threads != kMrgBlockThreads)
        return nullptr;
    return by_map(fam, [&](auto m) { return mrg_fill_kernel_for<decltype(m)::value>(fam, ppl, seq); });
}

// The wave-granular speculative fill of a single segment (or its repair)
// for a Philox-family generator; null for other families.
const void *spec_wave_kernel_for(uint32_t fam, bool repair, uint32_t windows)
{
    return by_map(fam, [&](auto m) {
        return philox_wave_kernel_for<decltype(m)::value>(fam, repair, windows);
    });
}

// The chunk-speculative batch fill (256 threads, chunks of `windows`
// 128-pair windows) or its repair (64 threads), or null.
const void *chunk_kernel_for(uint32_t fam, bool repair, uint32_t windows)
{
    return by_map(fam, [&](auto m) {
        return philox_chunk_kernel_for<decltype(m)::value>(fam, repair, windows);
    });
}

// The counted single fill: its counting or producing pass (256 threads),
// or null.
const void *counted_kernel_for(uint32_t fam, bool produce)
{
    return by_map(fam, [&](auto m) {
        return philox_counted_kernel_for<decltype(m)::value>(fam, produce);
    });
}

// A RANMAR kernel (256 threads; mode 0 one wave per request, 1 count, 2
// produce), for the map of family fam.
const void *ranmar_kernel_for(uint32_t fam, uint32_t mode)
{
    return by_map(fam, [&](auto m) { return ranmar_kernel_for<decltype(m)::value>(mode); });
}

// The two levels of its scan (1024 threads each).
const void *counted_scan_kernel_ptr(bool top)
{
    return top ? reinterpret_cast<const void *>(&counted_scan_top_kernel)
               : reinterpret_cast<const void *>(&counted_scan_blocks_kernel);
}

const void *chunk_prep_kernel_ptr()
{
    return reinterpret_cast<const void *>(&chunk_prep_kernel);
}

// The single-word-consumption kernel (256 threads), or null.
const void *single_kernel_for(uint32_t fam)
{
    return by_map(fam, [&](auto m) { return single_kernel_for<decltype(m)::value>(fam); });
}

// The one-word-consumption speculative fill of one segment across
// workgroups (256 threads), or its repair pass; null for other families.
const void *spec_words_kernel_for(uint32_t fam, bool repair)
{
    return by_map(fam, [&](auto m) { return spec_words_kernel_for<decltype(m)::value>(fam, repair); });
}

hipError_t launch_toggle_flip(uint32_t *flip, hipStream_t stream)
{
    hipLaunchKernelGGL(toggle_flip_kernel, dim3(1), dim3(1), 0, stream, flip);
    return hipGetLastError();
}

const void *toggle_flip_kernel_ptr()
{
    return reinterpret_cast<const void *>(&toggle_flip_kernel);
}

hipError_t launch_fill(const void *kernel, uint32_t grid, uint32_t threads, const LaunchArgs &args,
                       hipStream_t stream)
{
    void *params[] = {const_cast<LaunchArgs *>(&args)};
    return hipLaunchKernel(kernel, dim3(grid), dim3(threads), params, 0, stream);
}

hipError_t launch_set_counter(uint64_t *slot, uint64_t value, hipStream_t stream)
{
    hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(1), 0, stream, slot, value);
    return hipGetLastError();
}

hipError_t launch_ranmar_set(const RanmarInit &r, hipStream_t stream)
{
    hipLaunchKernelGGL(ranmar_set_state_kernel, dim3(1), dim3(128), 0, stream, r);
    return hipGetLastError();
}

hipError_t launch_ranmar_set_many(const RanmarInit *inits, uint32_t count, hipStream_t stream)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(ranmar_set_states_kernel, dim3(count), dim3(128), 0, stream, inits, count);
    return hipGetLastError();
}

hipError_t launch_zero_words(uint64_t *p, size_t n, hipStream_t stream)
{
    if (n == 0)
        return hipSuccess;
    const size_t blocks = (n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096;
    hipLaunchKernelGGL(zero_words_kernel, dim3(uint32_t(blocks)), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

hipError_t launch_expand_tiles(const Segment *segs, uint32_t nseg, uint32_t *tile_seg,
                               hipStream_t stream)
{
    if (nseg == 0)
        return hipSuccess;
    const uint32_t blocks = nseg < 8192 ? nseg : 8192;
    hipLaunchKernelGGL(expand_tiles_kernel, dim3(blocks), dim3(256), 0, stream, segs, nseg,
                       tile_seg);
    return hipGetLastError();
}

}  // namespace prngd
