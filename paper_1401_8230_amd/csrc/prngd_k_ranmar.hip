// prngd_k_ranmar.hip -- PRNGD fills on the words of RANMAR (Marsaglia,
// Zaman, Tsang 1990, one of the 24-bit generators Section 2 names as
// suitable).  Built twice: with PRNGD_MAPF = 0 (the Eq. (5) kernels) and
// PRNGD_MAPF = FAM_ANY_MAP.
//
// RANMAR is a lagged generator: its words come from a window of 97 lagged
// values, not from a counter.  A wave produces one stretch of a stream
// (a segment) from the window at the stretch's start, 64 lagged values a
// step into a ring of 512 values in the wave's own LDS (kept twice, so
// that no read wraps): with the recurrence applied twice, L[t] = L[t-97] -
// L[t-130] + L[t-66], every value of a step depends only on earlier steps
// (the first 33 values of a segment, whose L[t-33] is a start value, take
// the recurrence once).  Lagged values are kept mod 2^32; their low 24 bits
// are the generator's.  Then every lane takes two pairs (four words) of
// each 128-pair window, and the window is accepted, ranked and stored as
// the Philox windows are.  A segment's start window
// comes from the stream's start window by the jump x^(2 g P) mod (x^97 +
// x^64 - 1): window[s] = sum_i row[i] * L[W - 96 + s + i], 97 products per
// value, over the start window extended by 96 values.  A single long fill
// counts each segment's accepted pairs in one pass (mode 1), scans, and
// produces each segment at its offset (mode 2); the last segment continues
// until n outputs.  A batch gives each request one wave (mode 0).  The wave
// that stores output n - 1 writes the next pair counter and the window at
// the next position (into the other state slot).
#include "prngd_device.hpp"

namespace prngd {
namespace {

constexpr uint32_t kRing = 512;              // lagged values per wave (a power of two)
constexpr uint32_t kRingBase = 127;          // L[W + t] lives at ring[(kRingBase + t) % kRing],
                                             // and again kRing words on

// (C - d) mod CM for C, d in [0, CM)
__device__ __forceinline__ uint32_t csub(uint32_t c, uint32_t d)
{
    return c >= d ? c - d : c + kRanmarCM - d;
}

// Orders one wave's LDS accesses: writes before the fence are seen by the
// reads after it (the wave's LDS instructions complete in order; the fences
// keep the compiler from moving accesses across).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t ring_index(uint32_t t)
{
    return (kRingBase + t) & (kRing - 1);
}

// Store lagged value v at ring position p, in both copies.
__device__ __forceinline__ void ring_put(uint32_t *ring, uint32_t p, uint32_t v)
{
    ring[p] = v;
    ring[p + kRing] = v;
}

// Lagged values L[W + t0 + 1 .. W + t0 + count], 64 a step (t is taken
// mod 2^32, which the ring position ignores).  Lane l of a step makes
// L[W + t], t = t0 + s + 1 + l, reading the copy kRing words on at
// positions p + kRing - 97, - 130, - 66 (never below 0 nor past 2 kRing).
__device__ __forceinline__ void generate(uint32_t *ring, uint32_t t0, uint32_t count, uint32_t lane)
{
    for (uint32_t s = 0; s < count; s += 64u) {
        const uint32_t t = t0 + s + 1u + lane;
        if (s + lane < count) {
            const uint32_t p = ring_index(t);
            const uint32_t *q = ring + p + kRing;
            const uint32_t l97 = q[-97];
            uint32_t v;
            if (t0 + s == 0u && lane < 33u)
                v = l97 - q[-33];                     // L[t - 33] is a start value
            else
                v = l97 - q[-130] + q[-66];
            ring_put(ring, p, v);
        }
        wave_lds_sync();
    }
}

// (256 * 7654321) mod 16777213: C moves by this over one 128-pair window.
constexpr uint32_t kWindowC = uint32_t((uint64_t(256) * kRanmarCD) % kRanmarCM);

template <uint32_t FAM>
struct RanmarWave {
    using WC = WaveChunk<FAM>;
    using HiLo = typename WC::HiLo;

    // The four words of lane l in window m (relative words 256 m + 4 l ..
    // + 3, word j being L[W + j + 1] - C[W + j + 1]) as x1 - a0 - 1 and
    // x2 - b0 of its two pairs (a0 = b0 = 0).  cw = C[W + 256 m]; d[i] =
    // ((4 l + i + 1) * 7654321) mod 16777213.
    __device__ __forceinline__ static HiLo words(const uint32_t *ring, uint32_t m, uint32_t cw,
                                                 const uint32_t d[4], uint32_t lane)
    {
        const uint4 L = *reinterpret_cast<const uint4 *>(ring + ((kRingBase + 1u + 256u * m + 4u * lane) & (kRing - 1)));
        const uint32_t w0 = (L.x - csub(cw, d[0])) & kRanmarMask;
        const uint32_t w1 = (L.y - csub(cw, d[1])) & kRanmarMask;
        const uint32_t w2 = (L.z - csub(cw, d[2])) & kRanmarMask;
        const uint32_t w3 = (L.w - csub(cw, d[3])) & kRanmarMask;
        return {w0 - 1u, w1, w2 - 1u, w3};
    }
};

template <uint32_t FAM, int MODE>
__global__ __launch_bounds__(256) void ranmar_kernel(LaunchArgs args)
{
    using RW = RanmarWave<FAM>;
    using WC = WaveChunk<FAM>;
    __shared__ __align__(16) uint32_t s_ring[4][2 * kRing];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t k = blockIdx.x * 4u + wave;
    if (k >= args.total_tiles)
        return;                                   // no workgroup barrier below
    uint32_t *ring = s_ring[wave];
    const Segment seg = MODE == 0 && args.segs ? args.segs[k] : args.seg0;
    const uint32_t flip = ((constant_u32 *)args.flip)[0];
    const uint32_t par = (seg.parity ^ flip) & 1u;
    RanmarState *state = reinterpret_cast<RanmarState *>(seg.seed);
    const uint32_t *st_in = state->slot[par];
    uint32_t *st_out = state->slot[par ^ 1u];
    uint64_t *next_counter = seg.counter + (par ^ 1u);
    const uint64_t c0 = ((constant_u64 *)seg.counter)[par];

    // the window at the stream's start: ring[31 .. 127] = L[W - 96 .. W]
    ring_put(ring, kRingBase - 96u + lane, st_in[lane]);
    if (lane < 33)
        ring_put(ring, kRingBase - 32u + lane, st_in[64 + lane]);
    uint32_t cw = __builtin_amdgcn_readfirstlane(st_in[96 + 1]);
    wave_lds_sync();
    uint64_t pair_start = c0;
    if (MODE != 0 && k > 0) {
        // segment k starts 2 k P words on: its window from the start window
        // extended by 96 values, through row k of the jump table
        generate(ring, 0u, 96u, lane);
        const constant_u32 *row = (const constant_u32 *)(args.ranmar_jump + size_t(k) * kRanmarRow);
        uint32_t acc0 = 0, acc1 = 0;
#pragma unroll 8
        for (uint32_t i = 0; i < 97; ++i) {
            const uint32_t r = row[i];
            acc0 += uint32_t(__umul24(r, ring[kRingBase - 96u + lane + i]));
            acc1 += uint32_t(__umul24(r, ring[kRingBase - 32u + lane + i]));   // used by lanes < 33
        }
        wave_lds_sync();
        ring_put(ring, kRingBase - 96u + lane, acc0 & kRanmarMask);
        if (lane < 33)
            ring_put(ring, kRingBase - 32u + lane, acc1 & kRanmarMask);
        cw = csub(cw, row[97]);
        wave_lds_sync();
        pair_start = c0 + uint64_t(k) * args.ranmar_seg_pairs;
    }
    uint32_t d[4];
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i)
        d[i] = uint32_t((uint64_t(4u * lane + i + 1u) * kRanmarCD) % kRanmarCM);

    const uint32_t windows = MODE == 0 ? 0xFFFFFFFFu : args.ranmar_seg_pairs / kChunk;
    const bool last = MODE == 0 || k == args.total_tiles - 1;
    uint64_t excl = 0;
    if (MODE == 2)
        excl = __builtin_amdgcn_readfirstlane(args.block_offs[k / kScanBlock]) +
               __builtin_amdgcn_readfirstlane(args.chunk_offs[k]);
    uint32_t counted = 0;
    const uint32_t hm = args.a - args.a0 - 1u;
    // a bound no correct stream reaches (a window keeps 128 pairs but for
    // one in 2^23 on average), so that every wave ends
    const uint64_t cap = uint64_t(windows == 0xFFFFFFFFu ? 0u : windows) +
                         2u * ((seg.n - excl + kChunk - 1) / kChunk) + 64u;
    for (uint32_t m = 0;; ++m) {
        if (MODE == 1) {
            if (m == windows)
                break;
        } else if (!(m < windows || last) || !uniform_lt(excl, seg.n)) {
            break;
        } else if (!uniform_lt(m, cap)) {
            if (lane == 0)
                __hip_atomic_fetch_or(args.error, kErrRanmarRunaway, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_SYSTEM);
            break;
        }
        generate(ring, 256u * m, 256u, lane);
        const typename RW::HiLo p = RW::words(ring, m, cw, d, lane);
        if (MODE == 1) {
            counted += WC::emit(args, seg, p, 0, 0u, 0, nullptr, false, false);
            cw = csub(cw, kWindowC);
            continue;
        }
        const uint64_t pair0 = pair_start + uint64_t(kChunk) * m;
        const uint32_t kept = WC::emit(args, seg, p, pair0, 0u, excl, next_counter, true,
                                       chunk_fits(excl, seg.n));
        if (!uniform_lt(excl + kept, seg.n)) {
            // this window holds output n - 1: find its pair (as emit ranks
            // them) and leave the window and C after that pair
            const uint64_t ka = __builtin_amdgcn_ballot_w64(p.ha < hm);
            const uint64_t kb = __builtin_amdgcn_ballot_w64(p.hb < hm);
            const uint32_t r = uint32_t(seg.n - 1 - excl);
            const uint64_t lt = lanemask_lt(lane);
            const bool oka = (ka >> lane) & 1u, okb = (kb >> lane) & 1u;
            const uint32_t pos_a = uint32_t(__popcll(ka & lt) + __popcll(kb & lt));
            const uint32_t pos_b = pos_a + (oka ? 1u : 0u);
            const bool hit_a = oka && pos_a == r, hit_b = okb && pos_b == r;
            const uint64_t who = __builtin_amdgcn_ballot_w64(hit_a || hit_b);
            const uint32_t src = uint32_t(__builtin_ctzll(who));
            const uint32_t mine = 2u * lane + (hit_b ? 2u : 1u);   // pairs through output n - 1
            const uint32_t e = __builtin_amdgcn_readlane(mine, src);
            const uint32_t t_end = 256u * m + 2u * e;              // words consumed
            st_out[lane] = ring[ring_index(t_end - 96u + lane)] & kRanmarMask;
            if (lane < 33)
                st_out[64 + lane] = ring[ring_index(t_end - 32u + lane)] & kRanmarMask;
            if (lane == 0)
                st_out[97] = csub(cw, uint32_t((uint64_t(2u * e) * kRanmarCD) % kRanmarCM));
        }
        excl += kept;
        cw = csub(cw, kWindowC);
    }
    if (MODE == 1 && lane == 0)
        args.chunk_counts[k] = counted;
}

}  // namespace

template <>
const void *ranmar_kernel_for<PRNGD_MAPF>(uint32_t mode)
{
    constexpr uint32_t F = FAM_RANMAR | PRNGD_MAPF;
    switch (mode) {
    case 0: return reinterpret_cast<const void *>(&ranmar_kernel<F, 0>);
    case 1: return reinterpret_cast<const void *>(&ranmar_kernel<F, 1>);
    case 2: return reinterpret_cast<const void *>(&ranmar_kernel<F, 2>);
    default: return nullptr;
    }
}

}  // namespace prngd
