// prngd_kernels.hip -- gfx950 fill kernels of libprngd.
//
// One launch fills one or more segments (a segment = the next n outputs of
// one handle).  Each segment's pair range is cut into tiles of
// T = 256 * PPL consecutive pairs aligned to multiples of T; workgroups take
// tiles in ticket order, so a tile only ever waits for tiles that are
// already running.  Per tile:
//   1. base words in registers (Philox4x32-10, MRG32k3a, or the test
//      enumeration), the word transform x >> (32 - w);
//   2. accept/reject of x1 (Section 2 of the paper: x1 = a0 or x1 = a is
//      dropped, the pair is consumed);
//   3. the Eq. (5) map z' = RN(RN(N) * S), the only FP64 arithmetic;
//   4. order-preserving compaction: wave ballot + popcount, a block scan
//      in LDS, and a decoupled look-back over the segment's earlier tiles
//      for the tile's exclusive output offset;
//   5. coalesced stores, and the tile that writes output n - 1 stores the
//      handle's next pair counter.
// The last real tile of a segment continues past the planned pairs if
// rejections left the segment short ("take next pair" until n outputs).
#include <hip/hip_runtime.h>

#include "prngd_internal.hpp"

namespace prngd {
namespace {

typedef double double2v __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies; the high halves are XORed with the other counter
// words and the round key, the key advances by the Weyl constants.
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kWeyl0 = 0x9E3779B9u;
constexpr uint32_t kWeyl1 = 0xBB67AE85u;

struct Words4 {
    uint32_t v0, v1, v2, v3;
};

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = uint64_t(kPhiloxM0) * c0;
        const uint64_t p1 = uint64_t(kPhiloxM1) * c2;
        const uint32_t n0 = uint32_t(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = uint32_t(p0 >> 32) ^ c3 ^ k1;
        c1 = uint32_t(p1);
        c3 = uint32_t(p0);
        c0 = n0;
        c2 = n2;
        k0 += kWeyl0;
        k1 += kWeyl1;
    }
    return {c0, c1, c2, c3};
}

// -------------------------------------------------------------- MRG32k3a
// L'Ecuyer 1999.  Moduli m1 = 2^32 - 209, m2 = 2^32 - 22853; reductions
// fold the high word with 2^32 = c (mod m).
constexpr uint32_t kM1 = 4294967087u;
constexpr uint32_t kM2 = 4294944443u;

__device__ __forceinline__ uint32_t red_m1(uint64_t x)
{
    x = (x >> 32) * 209u + (x & 0xffffffffu);
    x = (x >> 32) * 209u + (x & 0xffffffffu);
    return uint32_t(x >= kM1 ? x - kM1 : x);
}

__device__ __forceinline__ uint32_t red_m2(uint64_t x)
{
    x = (x >> 32) * 22853u + (x & 0xffffffffu);
    x = (x >> 32) * 22853u + (x & 0xffffffffu);
    return uint32_t(x >= kM2 ? x - kM2 : x);
}

struct Mrg {
    uint32_t s[6];   // (x1[n-3], x1[n-2], x1[n-1], x2[n-3], x2[n-2], x2[n-1])

    __device__ __forceinline__ uint32_t next()
    {
        const uint32_t p1 = red_m1(uint64_t(1403580u) * s[1] + uint64_t(810728u) * (kM1 - s[0]));
        const uint32_t p2 = red_m2(uint64_t(527612u) * s[5] + uint64_t(1370589u) * (kM2 - s[3]));
        s[0] = s[1]; s[1] = s[2]; s[2] = p1;
        s[3] = s[4]; s[4] = s[5]; s[5] = p2;
        return p1 > p2 ? p1 - p2 : p1 - p2 + kM1;
    }

    // s <- M s for one table entry: 3x3 for component 1 then component 2.
    __device__ __forceinline__ void apply(const uint32_t *__restrict__ M)
    {
        uint32_t r[6];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            uint64_t acc1 = 0, acc2 = 0;
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                acc1 += red_m1(uint64_t(M[3 * i + l]) * s[l]);
                acc2 += red_m2(uint64_t(M[9 + 3 * i + l]) * s[3 + l]);
            }
            r[i] = red_m1(acc1);
            r[3 + i] = red_m2(acc2);
        }
#pragma unroll
        for (int i = 0; i < 6; ++i)
            s[i] = r[i];
    }
};

// ------------------------------------------------------------- the map
// Eq. (5) in integer units: N = (x1 - a0 - 1) 2^w + (x2 - b0) is rounded to
// FP64 once (the 2^w scaling of the high part is exact, so this is also
// what an FMA would give), multiplied by the folded constant S with one
// rounding, and forced below 1 when the product rounds up to 1.0.
__device__ __forceinline__ double prngd_map(uint32_t x1, uint32_t x2, const LaunchArgs &a,
                                            double two_w)
{
    const double hi = double(x1 - a.a0 - 1u);
    const double lo = double(x2 - a.b0);
    const double N = hi * two_w + lo;
    const double z = N * a.S;
    return z >= 1.0 ? 0x1.fffffffffffffp-1 : z;
}

// ------------------------------------------------------- wave utilities
__device__ __forceinline__ uint64_t lanemask_lt(uint32_t lane)
{
    return (uint64_t(1) << lane) - 1;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, uint32_t lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t u = __shfl_up(v, d, 64);
        if (lane >= uint32_t(d))
            v += u;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
        v += __shfl_xor(v, d, 64);
    return v;
}

// ------------------------------------------------ status words, tickets
__device__ __forceinline__ uint64_t pack_status(uint32_t epoch, uint32_t flag, uint64_t value)
{
    return (uint64_t(epoch) << 40) | (uint64_t(flag) << kValueBits) | value;
}

__device__ __forceinline__ void publish(uint64_t *status, uint32_t g, uint64_t word)
{
    __hip_atomic_store(&status[g], word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive output offset of tile g, the t-th tile of its segment, from the
// status words of tiles g - t .. g - 1.  Run by one whole wave.  Status
// words of another launch carry another epoch and read as "not ready".
// The spin is bounded; a stall (impossible when every earlier tile is
// running) raises the error word and the launch's abort flag, which makes
// every other waiting tile and every idle workgroup give up at once.
__device__ uint64_t look_back(uint64_t *status, uint32_t g, uint32_t t, uint32_t epoch,
                              Control *ctl, uint32_t *error, uint32_t lane)
{
    uint64_t excl = 0;
    uint32_t left = t;
    uint32_t top = g - 1;
    uint32_t polls = 0;
    for (;;) {
        const bool valid = lane < left;
        uint32_t state;
        uint64_t value;
        uint32_t first;
        for (;;) {
            uint64_t word = 0;
            if (valid)
                word = __hip_atomic_load(&status[top - lane], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t ep = uint32_t(word >> 40);
            const uint32_t fl = uint32_t(word >> kValueBits) & 3u;
            state = !valid ? 3u : (ep == epoch ? fl : 0u);
            value = word & kValueMask;
            const uint64_t stop = __ballot(state >= kFlagPrefix);
            const uint64_t notready = __ballot(state == 0u);
            first = stop ? uint32_t(__builtin_ctzll(stop)) : 64u;
            const uint64_t below = first >= 64 ? ~uint64_t(0) : ((uint64_t(1) << first) - 1);
            if (!(notready & below))
                break;
            ++polls;
            if ((polls & 255u) == 0 &&
                __hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                return excl;
            if (polls > (1u << 20)) {
                if (lane == 0) {
                    __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_fetch_or(error, kErrLookbackStall, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_SYSTEM);
                }
                return excl;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        const bool take = lane < first || (lane == first && state == kFlagPrefix);
        excl += wave_sum_u64(take ? value : 0);
        if (first < 64)
            return excl;
        left -= 64;
        top -= 64;
    }
}

__device__ __forceinline__ Segment load_segment(const LaunchArgs &args, uint32_t ticket)
{
    if (args.segs == nullptr)
        return args.seg0;
    uint32_t lo = 0, hi = args.nseg;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (args.segs[mid].tile_begin <= ticket)
            lo = mid;
        else
            hi = mid;
    }
    return args.segs[lo];
}

// Geometry of tile t of a segment whose fill starts at pair c0.
struct TileGeom {
    uint64_t win;        // window index: pairs [win * T, (win + 1) * T)
    uint64_t lo, hi;     // pairs of this fill inside the window
    uint32_t nreal;      // windows the planned range touches
};

template <uint64_t T>
__device__ __forceinline__ TileGeom tile_geom(uint64_t c0, uint64_t planned, uint32_t t)
{
    TileGeom g;
    const uint64_t w0 = c0 / T;
    const uint64_t end = c0 + planned;               // one past the last planned pair
    g.nreal = uint32_t((end - 1) / T - w0 + 1);
    g.win = w0 + t;
    const uint64_t ws = g.win * T;
    g.lo = ws > c0 ? ws : c0;
    g.hi = ws + T < end ? ws + T : end;
    return g;
}

__device__ __forceinline__ void store_one(double *p, double v, uint32_t mode)
{
    if (mode == 2)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

__device__ __forceinline__ void store_two(double *p, double v0, double v1, uint32_t mode)
{
    double2v v = {v0, v1};
    if (mode == 2)
        __builtin_nontemporal_store(v, reinterpret_cast<double2v *>(p));
    else
        *reinterpret_cast<double2v *>(p) = v;
}

__device__ __forceinline__ void finish_launch(const LaunchArgs &args, uint32_t epoch)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        Control *ctl = args.ctl;
        const uint32_t prev = __hip_atomic_fetch_add(&ctl->done, 1u, __ATOMIC_ACQ_REL,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        if (prev == gridDim.x - 1) {
            // every workgroup has taken its last ticket: reset for the next launch
            const uint32_t next = epoch >= kEpochMask ? 1u : epoch + 1u;
            __hip_atomic_store(&ctl->ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->epoch, next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->abort, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (args.use_flip)
                __hip_atomic_store(&ctl->flip, ctl->flip ^ 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Next tile ticket of this workgroup, or ~0 once the launch is aborted.
__device__ __forceinline__ uint32_t next_ticket(Control *ctl, uint32_t *s_ticket)
{
    if (threadIdx.x == 0) {
        const uint32_t t = __hip_atomic_fetch_add(&ctl->ticket, 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t ab = __hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        *s_ticket = ab ? ~0u : t;
    }
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(*s_ticket);
}

// ======================================================================
// Philox / enumerate family.  Thread (wave v, lane l) of the block takes
// Philox block  win * T / 2 + j * 256 + 64 v + l  for j < PPL / 2, i.e. the
// two consecutive pairs 2b, 2b + 1; for a fixed j a wave covers 128
// consecutive pairs, so its outputs are contiguous in memory.
// ======================================================================
template <int PPL, uint32_t FAM>
struct PhiloxTile {
    static constexpr int J = PPL / 2;
    static constexpr uint64_t T = uint64_t(kBlockThreads) * PPL;

    double v[PPL];
    uint32_t acc;          // bit i: pair i of this thread accepted

    // Generate, accept and map the pairs of window `win` restricted to
    // [lo, hi); leaves per-(j, wave) exclusive offsets in s_off and
    // returns the tile's accepted count.
    __device__ __forceinline__ uint32_t generate(const LaunchArgs &args, const Segment &seg,
                                                 uint64_t win, uint64_t lo, uint64_t hi,
                                                 uint32_t *s_off, uint32_t *s_total)
    {
        const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
        const uint32_t shift = 32u - args.w;
        const double two_w = double(uint64_t(1) << args.w);
        const uint64_t blk0 = win * (T / 2);
        const uint32_t k0 = uint32_t(seg.seed), k1 = uint32_t(seg.seed >> 32);
        acc = 0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const uint64_t slab = 2 * (blk0 + uint64_t(j) * kBlockThreads);   // first pair of slab j
            const uint64_t blk = blk0 + uint64_t(j) * kBlockThreads + tid;
            const uint64_t p = 2 * blk;
            uint32_t x1a, x2a, x1b, x2b;
            if (slab + 2 * kBlockThreads <= lo || slab >= hi) {
                x1a = x2a = x1b = x2b = args.a0;      // slab outside the fill
            } else if (FAM == FAM_PHILOX) {
                const Words4 r = philox4x32_10(uint32_t(blk), uint32_t(blk >> 32), 0u,
                                               seg.stream_id, k0, k1);
                x1a = r.v0 >> shift;
                x2a = r.v1 >> shift;
                x1b = r.v2 >> shift;
                x2b = r.v3 >> shift;
            } else {
                const uint64_t mask = (uint64_t(1) << args.w) - 1;
                x1a = uint32_t((p >> args.w) & mask);
                x2a = uint32_t(p & mask);
                x1b = uint32_t(((p + 1) >> args.w) & mask);
                x2b = uint32_t((p + 1) & mask);
            }
            const bool oka = p >= lo && p < hi && x1a != args.a0 && x1a != args.a;
            const bool okb = p + 1 >= lo && p + 1 < hi && x1b != args.a0 && x1b != args.a;
            v[2 * j] = prngd_map(x1a, x2a, args, two_w);
            v[2 * j + 1] = prngd_map(x1b, x2b, args, two_w);
            acc |= (uint32_t(oka) << (2 * j)) | (uint32_t(okb) << (2 * j + 1));
            const uint64_t ba = __ballot(oka), bb = __ballot(okb);
            if (lane == 0)
                s_off[j * kWavesPerBlock + wave] = uint32_t(__popcll(ba) + __popcll(bb));
        }
        __syncthreads();
        // exclusive scan over (j, wave) in pair order, by wave 0
        if (wave == 0) {
            const uint32_t e = lane;
            const uint32_t c = e < uint32_t(J * kWavesPerBlock) ? s_off[e] : 0u;
            const uint32_t inc = wave_incl_scan(c, lane);
            if (e < uint32_t(J * kWavesPerBlock))
                s_off[e] = inc - c;
            if (lane == 63)
                *s_total = inc;
        }
        __syncthreads();
        return *s_total;
    }

    // Store the accepted outputs of this tile at segment offset `excl`.
    __device__ __forceinline__ void store(const LaunchArgs &args, const Segment &seg,
                                          uint64_t win, uint64_t excl, uint64_t *next_counter,
                                          const uint32_t *s_off)
    {
        const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
        const uint64_t lt = lanemask_lt(lane);
        const uint64_t blk0 = win * (T / 2);
        const uint64_t n = seg.n;
        double *out = seg.out;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const bool oka = (acc >> (2 * j)) & 1u;
            const bool okb = (acc >> (2 * j + 1)) & 1u;
            const uint64_t ba = __ballot(oka), bb = __ballot(okb);
            const uint64_t pos_a = excl + s_off[j * kWavesPerBlock + wave] +
                                   uint32_t(__popcll(ba & lt) + __popcll(bb & lt));
            const uint64_t pos_b = pos_a + (oka ? 1u : 0u);
            const uint64_t pair = 2 * (blk0 + uint64_t(j) * kBlockThreads + tid);
            if (oka && okb && pos_b < n && args.store_mode != 1 &&
                ((reinterpret_cast<uintptr_t>(out + pos_a) & 15u) == 0)) {
                store_two(out + pos_a, v[2 * j], v[2 * j + 1], args.store_mode);
            } else {
                if (oka && pos_a < n)
                    store_one(out + pos_a, v[2 * j], args.store_mode);
                if (okb && pos_b < n)
                    store_one(out + pos_b, v[2 * j + 1], args.store_mode);
            }
            if (oka && pos_a == n - 1)
                *next_counter = pair + 1;
            if (okb && pos_b == n - 1)
                *next_counter = pair + 2;
        }
    }
};

// ======================================================================
// MRG32k3a / mixed family.  MRG32k3a is a recurrence, so each thread takes
// PPL consecutive pairs and steps its own state from a jump-ahead start;
// compacted outputs are staged in LDS and written out by consecutive
// threads so that the stores stay coalesced.
// ======================================================================
__device__ __forceinline__ uint32_t pad_index(uint32_t i)
{
    return i + (i >> 4);     // one spare slot per 16 doubles against bank conflicts
}

template <int PPL, uint32_t FAM>
struct MrgTile {
    static constexpr uint64_t T = uint64_t(kBlockThreads) * PPL;
    static constexpr uint32_t R = FAM == FAM_MRG ? 2u : 1u;   // MRG outputs per pair
    static_assert(PPL % 4 == 0, "Philox blocks must not straddle threads");

    double v[PPL];
    uint32_t acc;
    uint32_t thread_off;   // exclusive offset of this thread inside the tile

    __device__ __forceinline__ uint32_t generate(const LaunchArgs &args, const Segment &seg,
                                                 uint64_t win, uint64_t lo, uint64_t hi,
                                                 uint32_t *s_wave, uint32_t *s_total)
    {
        const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
        const double two_w = double(uint64_t(1) << args.w);
        const uint64_t p0 = win * T + uint64_t(tid) * PPL;
        acc = 0;
        if (p0 + PPL > lo && p0 < hi) {
            Mrg g;
#pragma unroll
            for (int i = 0; i < 6; ++i)
                g.s[i] = seg.mrg[i];
            // jump to MRG position R * p0 = R * T * win + R * PPL * tid
            uint64_t m = win;
            for (int d = 0; d < kMrgDigits && m != 0; ++d, m >>= 8) {
                const uint32_t digit = uint32_t(m & 255u);
                if (digit)
                    g.apply(args.mrg_window + (size_t(d) * 256 + digit) * kMrgMatWords);
            }
            g.apply(args.mrg_thread + size_t(tid) * kMrgMatWords);
            const uint32_t k0 = uint32_t(seg.seed), k1 = uint32_t(seg.seed >> 32);
            Words4 ph = {0, 0, 0, 0};
#pragma unroll
            for (int i = 0; i < PPL; ++i) {
                const uint64_t p = p0 + i;
                uint32_t x1, x2;
                if (FAM == FAM_MIXED) {
                    if ((i & 3) == 0) {
                        const uint64_t blk = p >> 2;
                        ph = philox4x32_10(uint32_t(blk), uint32_t(blk >> 32), 0u,
                                           seg.stream_id, k0, k1);
                    }
                    x1 = (i & 3) == 0 ? ph.v0 : (i & 3) == 1 ? ph.v1 : (i & 3) == 2 ? ph.v2 : ph.v3;
                    x2 = g.next();
                } else {
                    x1 = g.next();
                    x2 = g.next();
                }
                const bool ok = p >= lo && p < hi && x1 != args.a0 && x1 != args.a;
                v[i] = prngd_map(ok ? x1 : args.a0 + 1u, ok ? x2 : args.b0, args, two_w);
                acc |= uint32_t(ok) << i;
            }
        }
        const uint32_t c = uint32_t(__popc(acc));
        const uint32_t inc = wave_incl_scan(c, lane);
        if (lane == 63)
            s_wave[wave] = inc;
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int k = 0; k < kWavesPerBlock; ++k) {
            const uint32_t t = s_wave[k];
            before += uint32_t(k) < wave ? t : 0u;
            total += t;
        }
        thread_off = before + inc - c;
        __syncthreads();       // s_wave is reused by the next tile
        (void)s_total;
        return total;
    }

    __device__ __forceinline__ void store(const LaunchArgs &args, const Segment &seg,
                                          uint64_t win, uint64_t excl, uint32_t total,
                                          uint64_t *next_counter, double *s_vals)
    {
        const uint32_t tid = threadIdx.x;
        const uint64_t n = seg.n;
        const uint64_t p0 = win * T + uint64_t(tid) * PPL;
        uint32_t k = thread_off;
#pragma unroll
        for (int i = 0; i < PPL; ++i) {
            if ((acc >> i) & 1u) {
                s_vals[pad_index(k)] = v[i];
                if (excl + k == n - 1)
                    *next_counter = p0 + i + 1;
                ++k;
            }
        }
        __syncthreads();
        double *out = seg.out;
        for (uint32_t i = tid; i < total; i += kBlockThreads) {
            const uint64_t pos = excl + i;
            if (pos < n)
                store_one(out + pos, s_vals[pad_index(i)], args.store_mode == 1 ? 0u : args.store_mode);
        }
        __syncthreads();       // s_vals is reused by the next tile
    }
};

// ======================================================================
// Kernels.
// ======================================================================
template <int PPL, uint32_t FAM>
__global__ __launch_bounds__(kBlockThreads) void fill_philox_kernel(LaunchArgs args)
{
    using Tile = PhiloxTile<PPL, FAM>;
    constexpr uint64_t T = Tile::T;
    __shared__ uint32_t s_off[Tile::J * kWavesPerBlock];
    __shared__ uint32_t s_total;
    __shared__ uint64_t s_excl;
    __shared__ uint32_t s_ticket;

    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t epoch = args.ctl->epoch;
    const uint32_t flip = args.use_flip ? args.ctl->flip : 0u;

    for (;;) {
        const uint32_t ticket = next_ticket(args.ctl, &s_ticket);
        if (ticket >= args.total_tiles)
            break;
        const Segment seg = load_segment(args, ticket);
        const uint32_t t = ticket - seg.tile_begin;
        const uint32_t par = seg.parity ^ flip;
        const uint64_t c0 = seg.counter[par];
        uint64_t *next_counter = seg.counter + (par ^ 1u);
        const TileGeom geom = tile_geom<T>(c0, seg.planned, t);
        if (t < geom.nreal) {
            Tile tile;
            const uint32_t agg = tile.generate(args, seg, geom.win, geom.lo, geom.hi, s_off, &s_total);
            if (t == 0) {
                if (tid == 0) {
                    publish(args.status, ticket, pack_status(epoch, kFlagPrefix, agg));
                    s_excl = 0;
                }
            } else {
                if (tid == 0)
                    publish(args.status, ticket, pack_status(epoch, kFlagAggregate, agg));
                if (tid < 64) {
                    const uint64_t excl = look_back(args.status, ticket, t, epoch, args.ctl, args.error, lane);
                    if (tid == 0) {
                        publish(args.status, ticket, pack_status(epoch, kFlagPrefix, excl + agg));
                        s_excl = excl;
                    }
                }
            }
            __syncthreads();
            uint64_t running = s_excl;
            tile.store(args, seg, geom.win, running, next_counter, s_off);
            running += agg;
            // tail: the last real tile takes further pairs until n outputs
            if (t == geom.nreal - 1 && running < seg.n) {
                const uint64_t from = c0 + seg.planned;
                for (uint64_t win = from / T; running < seg.n; ++win) {
                    __syncthreads();
                    const uint32_t a2 = tile.generate(args, seg, win, from, ~uint64_t(0), s_off, &s_total);
                    tile.store(args, seg, win, running, next_counter, s_off);
                    running += a2;
                }
            }
        }
        __syncthreads();
    }
    finish_launch(args, epoch);
}

template <int PPL, uint32_t FAM>
__global__ __launch_bounds__(kBlockThreads) void fill_mrg_kernel(LaunchArgs args)
{
    using Tile = MrgTile<PPL, FAM>;
    constexpr uint64_t T = Tile::T;
    __shared__ double s_vals[T + T / 16];
    __shared__ uint32_t s_wave[kWavesPerBlock];
    __shared__ uint32_t s_total;
    __shared__ uint64_t s_excl;
    __shared__ uint32_t s_ticket;

    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t epoch = args.ctl->epoch;
    const uint32_t flip = args.use_flip ? args.ctl->flip : 0u;

    for (;;) {
        const uint32_t ticket = next_ticket(args.ctl, &s_ticket);
        if (ticket >= args.total_tiles)
            break;
        const Segment seg = load_segment(args, ticket);
        const uint32_t t = ticket - seg.tile_begin;
        const uint32_t par = seg.parity ^ flip;
        const uint64_t c0 = seg.counter[par];
        uint64_t *next_counter = seg.counter + (par ^ 1u);
        const TileGeom geom = tile_geom<T>(c0, seg.planned, t);
        if (t < geom.nreal) {
            Tile tile;
            const uint32_t agg = tile.generate(args, seg, geom.win, geom.lo, geom.hi, s_wave, &s_total);
            if (t == 0) {
                if (tid == 0) {
                    publish(args.status, ticket, pack_status(epoch, kFlagPrefix, agg));
                    s_excl = 0;
                }
            } else {
                if (tid == 0)
                    publish(args.status, ticket, pack_status(epoch, kFlagAggregate, agg));
                if (tid < 64) {
                    const uint64_t excl = look_back(args.status, ticket, t, epoch, args.ctl, args.error, lane);
                    if (tid == 0) {
                        publish(args.status, ticket, pack_status(epoch, kFlagPrefix, excl + agg));
                        s_excl = excl;
                    }
                }
            }
            __syncthreads();
            uint64_t running = s_excl;
            tile.store(args, seg, geom.win, running, agg, next_counter, s_vals);
            running += agg;
            if (t == geom.nreal - 1 && running < seg.n) {
                const uint64_t from = c0 + seg.planned;
                for (uint64_t win = from / T; running < seg.n; ++win) {
                    const uint32_t a2 = tile.generate(args, seg, win, from, ~uint64_t(0), s_wave, &s_total);
                    tile.store(args, seg, win, running, a2, next_counter, s_vals);
                    running += a2;
                }
            }
        }
        __syncthreads();
    }
    finish_launch(args, epoch);
}

// Sets a handle's position slot (both halves, so either parity reads it).
__global__ void set_counter_kernel(uint64_t *slot, uint64_t value)
{
    slot[0] = value;
    slot[1] = value;
}

__global__ void zero_words_kernel(uint64_t *p, size_t n)
{
    for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
         i += size_t(gridDim.x) * blockDim.x)
        p[i] = 0;
}

}  // namespace

// ---------------------------------------------------------------- dispatch
using KernelFn = void (*)(LaunchArgs);

template <int PPL>
static const void *philox_family(uint32_t fam)
{
    return fam == FAM_ENUM ? reinterpret_cast<const void *>(&fill_philox_kernel<PPL, FAM_ENUM>)
                           : reinterpret_cast<const void *>(&fill_philox_kernel<PPL, FAM_PHILOX>);
}

template <int PPL>
static const void *mrg_family(uint32_t fam)
{
    return fam == FAM_MRG ? reinterpret_cast<const void *>(&fill_mrg_kernel<PPL, FAM_MRG>)
                          : reinterpret_cast<const void *>(&fill_mrg_kernel<PPL, FAM_MIXED>);
}

// The kernel for (family, pairs per lane), or null if not instantiated.
const void *fill_kernel_for(uint32_t fam, uint32_t ppl)
{
    if (fam == FAM_PHILOX || fam == FAM_ENUM) {
        switch (ppl) {
        case 4: return philox_family<4>(fam);
        case 8: return philox_family<8>(fam);
        case 16: return philox_family<16>(fam);
        case 32: return philox_family<32>(fam);
        default: return nullptr;
        }
    }
    switch (ppl) {
    case 4: return mrg_family<4>(fam);
    case 8: return mrg_family<8>(fam);
    case 16: return mrg_family<16>(fam);
    default: return nullptr;
    }
}

hipError_t launch_fill(const void *kernel, uint32_t grid, const LaunchArgs &args, hipStream_t stream)
{
    void *params[] = {const_cast<LaunchArgs *>(&args)};
    return hipLaunchKernel(kernel, dim3(grid), dim3(kBlockThreads), params, 0, stream);
}

hipError_t launch_set_counter(uint64_t *slot, uint64_t value, hipStream_t stream)
{
    hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(1), 0, stream, slot, value);
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

}  // namespace prngd
