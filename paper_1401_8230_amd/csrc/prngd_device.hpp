// prngd_device.hpp -- gfx950 device code of libprngd's fill kernels,
// included by the kernel translation units (prngd_k_*.hip), each of which
// instantiates one family of kernels.
//
// One launch fills one or more segments (a segment = the next n outputs of
// one handle).  A segment's pairs are cut into windows of T = B * PPL
// consecutive pairs aligned to multiples of T (B threads per workgroup,
// PPL pairs per thread); tile t of a segment is its t-th window, the first
// one clipped at the start position.  Workgroups draw tiles in ticket
// order, so a tile only ever waits for tiles that are already running.
// Per tile:
//   1. base words in registers (Philox4x32-10, MRG32k3a, or the test
//      enumeration), the word transform x >> (32 - w);
//   2. accept/reject of x1 (Section 2 of the paper: x1 = a0 or x1 = a is
//      dropped, the pair is consumed);
//   3. the Eq. (5) map z' = RN(RN(N) * S), the only FP64 arithmetic;
//   4. order-preserving compaction: wave ballot + popcount, a block scan
//      in LDS, and a decoupled look-back over the segment's earlier tiles
//      for the tile's exclusive output offset;
//   5. coalesced stores; the thread that writes output n - 1 stores the
//      handle's next pair counter.
// The segment's last tile continues window by window until n outputs
// exist (every rejection moves the end of the segment one pair further).
#pragma once

#include <hip/hip_runtime.h>

#include "prngd_internal.hpp"

namespace prngd {
namespace {

typedef double double2v __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies; the high halves are XORed with the other counter
// words and the round key, the key advances by the Weyl constants.  Each
// three-way XOR is one gfx950 v_bitop3_b32 (truth table 0x96 = a ^ b ^ c),
// and each 32x32->64 product one v_mad_u64_u32.
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
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(uint32_t(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(uint32_t(p0 >> 32), c3, k1, 0x96);
        c1 = uint32_t(p1);
        c3 = uint32_t(p0);
        c0 = n0;
        c2 = n2;
        k0 += kWeyl0;
        k1 += kWeyl1;
    }
    return {c0, c1, c2, c3};
}

// A block per lane (counter c) and a block that is the same on every lane
// of the wave (counter u), with the rounds of the second on the scalar unit
// interleaved with those of the first so that the two issue side by side.
__device__ __forceinline__ void philox4x32_10_lane_and_uniform(const Words4 c, Words4 u,
                                                               uint32_t k0, uint32_t k1,
                                                               Words4 *rc, Words4 *ru)
{
    uint32_t c0 = c.v0, c1 = c.v1, c2 = c.v2, c3 = c.v3;
    uint32_t u0 = __builtin_amdgcn_readfirstlane(u.v0);
    uint32_t u1 = __builtin_amdgcn_readfirstlane(u.v1);
    uint32_t u2 = __builtin_amdgcn_readfirstlane(u.v2);
    uint32_t u3 = __builtin_amdgcn_readfirstlane(u.v3);
    k0 = __builtin_amdgcn_readfirstlane(k0);
    k1 = __builtin_amdgcn_readfirstlane(k1);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = uint64_t(kPhiloxM0) * c0;
        const uint64_t p1 = uint64_t(kPhiloxM1) * c2;
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(uint32_t(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(uint32_t(p0 >> 32), c3, k1, 0x96);
        c1 = uint32_t(p1);
        c3 = uint32_t(p0);
        c0 = n0;
        c2 = n2;
        const uint64_t q0 = uint64_t(kPhiloxM0) * u0;
        const uint64_t q1 = uint64_t(kPhiloxM1) * u2;
        const uint32_t m0 = uint32_t(q1 >> 32) ^ u1 ^ k0;
        const uint32_t m2 = uint32_t(q0 >> 32) ^ u3 ^ k1;
        u1 = uint32_t(q1);
        u3 = uint32_t(q0);
        u0 = m0;
        u2 = m2;
        k0 += kWeyl0;
        k1 += kWeyl1;
    }
    *rc = Words4{c0, c1, c2, c3};
    *ru = Words4{u0, u1, u2, u3};
}

// -------------------------------------------------------------- MRG32k3a
// L'Ecuyer 1999.  Moduli m1 = 2^32 - 209, m2 = 2^32 - 22853.  Reductions
// fold the high word with 2^32 = c (mod m), as many times as the operand's
// bound needs, and finish with one conditional subtraction of m, written
// as an addition of c in 32 bits (f - m = f + c - 2^32 for m <= f < 2 m).
constexpr uint32_t kM1 = 4294967087u;
constexpr uint32_t kM2 = 4294944443u;
constexpr uint32_t kC1 = 209u;      // 2^32 - m1
constexpr uint32_t kC2 = 22853u;    // 2^32 - m2

__device__ __forceinline__ uint64_t fold(uint64_t x, uint32_t c)
{
    return uint64_t(uint32_t(x >> 32)) * c + uint32_t(x);
}

// f mod m for f < 2 m
template <uint32_t M>
__device__ __forceinline__ uint32_t below_2m(uint64_t f)
{
    return f >= M ? uint32_t(f) + (0u - M) : uint32_t(f);
}

// x mod m1 for x < 2^54: one fold leaves f < 2^22 * 209 + 2^32 < 2 m1.
__device__ __forceinline__ uint32_t red_m1_54(uint64_t x)
{
    return below_2m<kM1>(fold(x, kC1));
}

// x mod m2 for x < 2^54: one fold leaves f < 2^36.5 + 2^32, a second
// f' < 17 * 22853 + 2^32 < 2 m2.
__device__ __forceinline__ uint32_t red_m2_54(uint64_t x)
{
    return below_2m<kM2>(fold(fold(x, kC2), kC2));
}

// (M0 s0 + M1 s1 + M2 s2) mod m for entries and state words below m: each
// product folded once (< 2^32 c + 2^32), the three summed (< 2^34 c), and
// the sum folded to below 2 m (m1: once, < 2^18 + 2^32; m2: twice).
template <uint32_t C>
__device__ __forceinline__ uint32_t dot3_mod(const uint32_t *__restrict__ M, uint32_t s0,
                                             uint32_t s1, uint32_t s2)
{
    const uint64_t acc = fold(uint64_t(M[0]) * s0, C) + fold(uint64_t(M[1]) * s1, C) +
                         fold(uint64_t(M[2]) * s2, C);
    if (C == kC1)
        return below_2m<kM1>(fold(acc, C));
    return below_2m<kM2>(fold(fold(acc, C), C));
}

struct Mrg {
    uint32_t s[6];   // (x1[n-3], x1[n-2], x1[n-1], x2[n-3], x2[n-2], x2[n-1])

    // The multipliers are below 2^21, so each sum of two products is below
    // 2^54.
    __device__ __forceinline__ uint32_t next()
    {
        const uint32_t p1 = red_m1_54(uint64_t(1403580u) * s[1] + uint64_t(810728u) * (kM1 - s[0]));
        const uint32_t p2 = red_m2_54(uint64_t(527612u) * s[5] + uint64_t(1370589u) * (kM2 - s[3]));
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
            r[i] = dot3_mod<kC1>(M + 3 * i, s[0], s[1], s[2]);
            r[3 + i] = dot3_mod<kC2>(M + 9 + 3 * i, s[3], s[4], s[5]);
        }
#pragma unroll
        for (int i = 0; i < 6; ++i)
            s[i] = r[i];
    }
};

// ------------------------------------------------------------- the map
// Eq. (5) in integer units: N = (x1 - a0 - 1) 2^w + (x2 - b0) is rounded to
// FP64 once -- the fused multiply-add of the exact product hi * 2^w and lo
// rounds once, exactly like converting the 64-bit integer N -- multiplied
// by the folded constant S with one rounding, and forced below 1: the
// largest double below 1 is the only value between a product that rounded
// up to 1.0 and every product that did not.  Eq. (4) (Algorithm 1's Z) is
// the same with N + 2^w - (b - b0) (lo + nadd stays exact: both are below
// 2^34) and S = RN(1 / D4); the no-zero form returns 1 - z, one rounding
// of the exact difference (fma(-1, z, 1)).  Kernels of a family without
// FAM_ANY_MAP compute Eq. (5) alone; the others take (nadd, S, osign,
// ooff) from the launch, and with Eq. (5)'s (0, S, 1, 0) they give the same
// bits.
constexpr double kBelowOne = 0x1.fffffffffffffp-1;

template <uint32_t FAM>
__device__ __forceinline__ double map_hi_lo(uint32_t hi, uint32_t lo, double two_w,
                                            const LaunchArgs &a)
{
    if (!(FAM & FAM_ANY_MAP)) {
        // Eq. (5): one fma, one multiply, one min
        const double z = __builtin_fma(double(hi), two_w, double(lo)) * a.S;
        return z < kBelowOne ? z : kBelowOne;
    }
    const double N = __builtin_fma(double(hi), two_w, double(lo) + a.nadd);
    const double z = N * a.S;
    return __builtin_fma(a.osign, z < kBelowOne ? z : kBelowOne, a.ooff);
}

template <uint32_t FAM>
__device__ __forceinline__ double prngd_map(uint32_t x1, uint32_t x2, const LaunchArgs &a,
                                            double two_w)
{
    return map_hi_lo<FAM>(x1 - a.a0 - 1u, x2 - a.b0, two_w, a);
}

// ------------------------------------------------------- wave utilities
// Lane i receives lane i - 1's value (lane 0 receives 0): one DPP
// wave_shr:1 move per 32-bit half, no LDS round trip.
__device__ __forceinline__ double wave_shr1(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b)), 0x138, 0xF, 0xF, false));
    const uint32_t hi = uint32_t(__builtin_amdgcn_update_dpp(0, int(uint32_t(b >> 32)), 0x138, 0xF, 0xF, false));
    return __builtin_bit_cast(double, uint64_t(hi) << 32 | lo);
}

// Lane i receives lane i + 1's value and lane 63 keeps `fill`: one DPP
// wave_shl:1 move whose invalid source lane leaves the old value in place.
__device__ __forceinline__ uint32_t wave_shl1_fill(uint32_t v, uint32_t fill)
{
    return uint32_t(__builtin_amdgcn_update_dpp(int(fill), int(v), 0x130, 0xF, 0xF, false));
}

// Lane i receives lane i + 1's value, lane 63 lane 0's (DPP wave_rol:1).
__device__ __forceinline__ uint32_t wave_rol1(uint32_t v)
{
    return uint32_t(__builtin_amdgcn_update_dpp(0, int(v), 0x134, 0xF, 0xF, false));
}

__device__ __forceinline__ uint64_t lanemask_lt(uint32_t lane)
{
    return (uint64_t(1) << lane) - 1;
}

// Whether p holds in any thread of the workgroup, as a value the compiler
// knows to be uniform: the block vote returns it through LDS, which would
// make every branch and loop that depends on it divergent (exec-mask
// bookkeeping on the scalar unit, loop state in vector registers).
__device__ __forceinline__ bool block_any(bool p)
{
    return __builtin_amdgcn_readfirstlane(uint32_t(__syncthreads_or(p))) != 0u;
}

// A workgroup-uniform value read back from LDS, marked uniform.
__device__ __forceinline__ uint32_t uniform_u32(uint32_t v)
{
    return __builtin_amdgcn_readfirstlane(v);
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

// Exclusive scan of cnt[0 .. E) in place by wave 0 (E <= 64 * K); the
// total lands in cnt[E].
template <int E>
__device__ __forceinline__ void wave0_scan(uint32_t *cnt, uint32_t lane)
{
    constexpr int K = (E + 63) / 64;
    uint32_t loc[K];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint32_t idx = lane * K + k;
        loc[k] = idx < uint32_t(E) ? cnt[idx] : 0u;
        sum += loc[k];
    }
    const uint32_t inc = wave_incl_scan(sum, lane);
    uint32_t run = inc - sum;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const uint32_t idx = lane * K + k;
        if (idx < uint32_t(E))
            cnt[idx] = run;
        run += loc[k];
    }
    if (lane == 63)
        cnt[E] = inc;
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
// The spin is bounded (`limit` polls); a stall (impossible when every
// earlier tile is running and the limit is the default) raises the error
// word and the launch's abort flag, which makes every other waiting tile
// and every idle workgroup give up at once.
__device__ inline uint64_t look_back(uint64_t *status, uint32_t g, uint32_t t, uint32_t epoch,
                              Control *ctl, uint32_t *error, uint32_t lane, uint32_t limit)
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
            if (polls > limit) {
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

// Launch-wide values every workgroup of the look-back kernel reads once at
// its start.
struct LaunchState {
    uint64_t base;
    uint32_t epoch;
    uint32_t flip;
};

__device__ __forceinline__ uint32_t read_flip(const LaunchArgs &args)
{
    return args.flip ? *args.flip : 0u;
}

__device__ __forceinline__ LaunchState read_launch_state(const LaunchArgs &args,
                                                         LaunchState *s_state)
{
    if (threadIdx.x == 0) {
        // acquire: this read completes before this workgroup draws tickets
        LaunchState st;
        st.base = __hip_atomic_load(&args.ctl->base, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        st.epoch = __hip_atomic_load(&args.ctl->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        st.flip = read_flip(args);
        *s_state = st;
    }
    __syncthreads();
    return *s_state;
}

// Tickets are drawn by thread 0 in two halves: issue() sends the atomic
// without waiting for it, finish() turns the result into a launch-local
// tile index, or ~0u when the launch has no tiles left.  The draw of the
// launch's very last ticket moves the control block on for the next
// launch.
__device__ __forceinline__ uint64_t issue_ticket(const LaunchArgs &args)
{
    return __hip_atomic_fetch_add(&args.ctl->ticket, uint64_t(1), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t finish_ticket(const LaunchArgs &args, const LaunchState &st,
                                                  uint64_t tk)
{
    Control *ctl = args.ctl;
    const uint64_t local = tk - st.base;
    const uint64_t total = args.total_tiles;
    if (local == total + gridDim.x - 1) {
        const uint32_t next = st.epoch >= kEpochMask ? 1u : st.epoch + 1u;
        __hip_atomic_store(&ctl->base, st.base + total + gridDim.x, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->epoch, next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->abort, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return local < total ? uint32_t(local) : ~0u;
}

// Descriptors, the tile map and the start positions are read-only while a
// launch runs (a fill writes only the other half of each position slot),
// so they are read through the constant address space: uniform scalar
// loads into SGPRs instead of vector loads into VGPRs.
typedef __attribute__((address_space(4))) const uint32_t constant_u32;
typedef __attribute__((address_space(4))) const uint64_t constant_u64;

__device__ __forceinline__ Segment load_segment(const Segment *segs, uint32_t i)
{
    static_assert(sizeof(Segment) % 8 == 0, "Segment is read as 64-bit words");
    constexpr int kWords = sizeof(Segment) / 8;
    const constant_u64 *src = (const constant_u64 *)(segs + i);
    uint64_t w[kWords];
#pragma unroll
    for (int k = 0; k < kWords; ++k)
        w[k] = src[k];
    Segment s;
    __builtin_memcpy(&s, w, sizeof s);
    return s;
}

__device__ __forceinline__ uint64_t load_start(const Segment &seg, uint32_t par)
{
    return ((constant_u64 *)seg.counter)[par];
}

__device__ __forceinline__ void lookup(const LaunchArgs &args, uint32_t local, Segment *seg,
                                       uint32_t *t)
{
    if (args.segs == nullptr) {
        *seg = args.seg0;
        *t = local;
    } else {
        const uint32_t si = ((constant_u32 *)args.tile_seg)[local];
        *seg = load_segment(args.segs, si);
        *t = local - seg->tile_begin;
    }
}

typedef __attribute__((address_space(1))) double global_double;
typedef __attribute__((address_space(1))) double2v global_double2;

__device__ __forceinline__ void store_one(double *p, double v, uint32_t mode)
{
    global_double *g = (global_double *)p;
    if (mode == 2)
        __builtin_nontemporal_store(v, g);
    else
        *g = v;
}

__device__ __forceinline__ void store_two(double *p, double v0, double v1, uint32_t mode)
{
    const double2v v = {v0, v1};
    global_double2 *g = (global_double2 *)p;
    if (mode == 2)
        __builtin_nontemporal_store(v, g);
    else
        *g = v;
}

// LDS index of staged value i: one spare slot per 16 doubles against bank
// conflicts.
__device__ __forceinline__ uint32_t pad_index(uint32_t i)
{
    return i + (i >> 4);
}

// Stores outputs [e0, e0 + cnt) of `out` that lie below n -- output e0 + i
// staged at s_vals[pad_index(i)] -- in 16-byte stores laid on the absolute
// 4 KB grid of addresses, so that each pass of a 256-thread workgroup
// writes one whole aligned 4 KB block (on MI355X plain streaming stores
// that straddle 128-byte lines ran up to 1.5x slower, and ones that
// straddle 4 KB blocks up to 1.13x).  Every thread of the B-thread
// workgroup calls it; store_mode 1 splits the 16-byte stores.
template <int B>
__device__ __forceinline__ void store_staged(double *out, uint64_t e0, uint32_t cnt, uint64_t n,
                                             const double *s_vals, uint32_t mode)
{
    const uint64_t a0 = reinterpret_cast<uintptr_t>(out + e0) >> 3;   // 8-byte slot of output e0
    const uint32_t r = uint32_t(a0 & 511u);        // slots of its 4 KB block before it
    const uint32_t slots = (cnt + r + 1u) >> 1;    // 16-byte slots from that block's start
    const uint32_t end = n <= e0 ? 0u : (n - e0 < cnt ? uint32_t(n - e0) : cnt);
    const uint32_t m1 = mode == 1 ? 0u : mode;
    double *o = out + e0;
    for (uint32_t base = 0; base < slots; base += B) {
        const uint32_t k = base + threadIdx.x;
        const int64_t i = int64_t(2u * k) - int64_t(r);   // range index of the slot's first output
        if (mode != 1 && 2u * base >= r &&
            int64_t(2u * (base + B)) - int64_t(r) <= int64_t(end)) {
            // every slot of this round lies inside the range
            store_two(o + i, s_vals[pad_index(uint32_t(i))], s_vals[pad_index(uint32_t(i + 1))],
                      m1);
            continue;
        }
        if (k >= slots)
            continue;
        const bool in0 = i >= 0 && i < int64_t(end);
        const bool in1 = i + 1 >= 0 && i + 1 < int64_t(end);
        if (in0 && in1 && mode != 1) {
            store_two(out + (e0 + uint64_t(i)), s_vals[pad_index(uint32_t(i))],
                      s_vals[pad_index(uint32_t(i + 1))], m1);
        } else {
            if (in0)
                store_one(out + (e0 + uint64_t(i)), s_vals[pad_index(uint32_t(i))], m1);
            if (in1)
                store_one(out + (e0 + uint64_t(i + 1)), s_vals[pad_index(uint32_t(i + 1))], m1);
        }
    }
}

// ======================================================================
// Philox / enumerate family.  A window is T consecutive pairs from an even
// pair wb (a Philox block boundary); thread tid of the B-thread workgroup
// takes Philox block  wb / 2 + j * B + tid  for j < PPL / 2, i.e. the two
// consecutive pairs at window offsets q = 2 (j B + tid) and q + 1; for a
// fixed j a wave covers 128 consecutive pairs, so its outputs are
// contiguous in memory.
//
// A window is "clean" when it starts at offset 0 and keeps every pair --
// at w = 32 all but a fraction 2^-31 of windows.  Its outputs are then
// consecutive from the window's offset and need neither ranks nor a scan;
// only windows with a rejection or a clipped start take the general path
// (ballots, per-(j, wave) counts, an LDS scan).
// ======================================================================
template <int NW, int PPL, uint32_t FAM>
struct PhiloxTile {
    static constexpr int B = 64 * NW;
    static constexpr int J = PPL / 2;
    static constexpr uint32_t T = uint32_t(B) * PPL;
    static constexpr int E = J * NW;           // (j, wave) groups in pair order
    static constexpr uint32_t kAll = PPL == 32 ? 0xFFFFFFFFu : ((1u << PPL) - 1u);

    double v[PPL];
    uint32_t acc;                              // bit i: pair i of this thread kept
    bool clean;                                // every pair of the window kept
    bool runs;                                 // wave-contiguous layout (odd wb)

    // LDS words the caller provides as s_off.
    static constexpr int kOffWords = E + 1;

    // Window offset of this thread's first pair in slot j, and the index of
    // its (j, wave) group in pair order.  Normally a wave covers 128
    // consecutive pairs per j (q = 2 (j B + tid)); in the wave-contiguous
    // layout wave w covers pairs [128 J w, 128 J (w + 1)), 128 per j.
    __device__ __forceinline__ uint32_t pair_q(int j) const
    {
        const uint32_t tid = threadIdx.x;
        return runs ? 2u * ((tid >> 6) * (64u * J) + uint32_t(j) * 64u + (tid & 63u))
                    : 2u * (uint32_t(j) * B + tid);
    }
    __device__ __forceinline__ uint32_t group(int j) const
    {
        const uint32_t wave = threadIdx.x >> 6;
        return runs ? wave * J + uint32_t(j) : uint32_t(j) * NW + wave;
    }

    // Generate the window of T pairs from pair wb, from window offset lo_off
    // on, and return its number of accepted pairs; for a window that is not
    // clean the exclusive offset of every (j, wave) group is left in s_off
    // (kOffWords words).  A window may start on the second pair of a Philox
    // block (odd wb): each thread then takes its block's second pair and the
    // first pair of the block after it.  With wave-contiguous blocks that is
    // the next lane's block, or for lane 63 lane 0's block of the next slot,
    // or the block after the wave's run, which each wave computes once.
    __device__ __forceinline__ uint32_t generate(const LaunchArgs &args, const Segment &seg,
                                                 uint64_t wb, uint32_t lo_off, uint32_t *s_off)
    {
        const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
        const uint64_t blk0 = (wb >> 1);
        const uint32_t k0 = uint32_t(seg.seed), k1 = uint32_t(seg.seed >> 32);
        acc = 0;
        runs = fam_base(FAM) != FAM_ENUM && (wb & 1u);
        if (runs) {
            uint32_t a1[J], a2[J], b1[J], b2[J];
            const uint64_t run0 = blk0 + uint64_t(wave) * (64u * J);
            // J blocks per lane on the vector unit and the block after the
            // run, the same for every lane of the wave, on the scalar unit:
            // its rounds are interleaved with the vector rounds so that they
            // issue beside them
            uint32_t c0[J], c1[J], c2[J], c3[J];
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const uint64_t blk = run0 + uint32_t(j) * 64u + lane;
                c0[j] = uint32_t(blk);
                c1[j] = uint32_t(blk >> 32);
                c2[j] = 0u;
                c3[j] = seg.stream_id;
            }
            const uint64_t nb = run0 + 64u * J;
            uint32_t u0 = __builtin_amdgcn_readfirstlane(uint32_t(nb));
            uint32_t u1 = __builtin_amdgcn_readfirstlane(uint32_t(nb >> 32));
            uint32_t u2 = 0u;
            uint32_t u3 = __builtin_amdgcn_readfirstlane(seg.stream_id);
            uint32_t r0 = __builtin_amdgcn_readfirstlane(k0);
            uint32_t r1 = __builtin_amdgcn_readfirstlane(k1);
#pragma unroll
            for (int r = 0; r < 10; ++r) {
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    const uint64_t p0 = uint64_t(kPhiloxM0) * c0[j];
                    const uint64_t p1 = uint64_t(kPhiloxM1) * c2[j];
                    const uint32_t n0 = __builtin_amdgcn_bitop3_b32(uint32_t(p1 >> 32), c1[j], r0, 0x96);
                    const uint32_t n2 = __builtin_amdgcn_bitop3_b32(uint32_t(p0 >> 32), c3[j], r1, 0x96);
                    c1[j] = uint32_t(p1);
                    c3[j] = uint32_t(p0);
                    c0[j] = n0;
                    c2[j] = n2;
                }
                const uint64_t q0 = uint64_t(kPhiloxM0) * u0;
                const uint64_t q1 = uint64_t(kPhiloxM1) * u2;
                const uint32_t m0 = uint32_t(q1 >> 32) ^ u1 ^ r0;
                const uint32_t m2 = uint32_t(q0 >> 32) ^ u3 ^ r1;
                u1 = uint32_t(q1);
                u3 = uint32_t(q0);
                u0 = m0;
                u2 = m2;
                r0 += kWeyl0;
                r1 += kWeyl1;
            }
#pragma unroll
            for (int j = 0; j < J; ++j) {
                a1[j] = c2[j];
                a2[j] = c3[j];
                b1[j] = c0[j];      // this block's first pair goes to the lane before
                b2[j] = c1[j];
            }
            const Words4 rn{u0, u1, u2, u3};
            // each lane's second pair is lane + 1's first; lane 63's is lane
            // 0's of the next slot (a rotation leaves it in lane 63) or the
            // first pair of the block after the run
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const uint32_t f1 = j + 1 < J ? wave_rol1(b1[j + 1 < J ? j + 1 : j]) : rn.v0;
                const uint32_t f2 = j + 1 < J ? wave_rol1(b2[j + 1 < J ? j + 1 : j]) : rn.v1;
                b1[j] = wave_shl1_fill(b1[j], f1);
                b2[j] = wave_shl1_fill(b2[j], f2);
            }
            if (fam_base(FAM) == FAM_PHILOX32) {
                // x in [0, 2^32 - 1]: as for windows on a block boundary
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    const bool oka = a1[j] + 1u >= 2u;
                    const bool okb = b1[j] + 1u >= 2u;
                    v[2 * j] = map_hi_lo<FAM>(a1[j] - 1u, a2[j], 4294967296.0, args);
                    v[2 * j + 1] = map_hi_lo<FAM>(b1[j] - 1u, b2[j], 4294967296.0, args);
                    acc |= (uint32_t(oka) << (2 * j)) | (uint32_t(okb) << (2 * j + 1));
                }
            } else {
                const uint32_t shift = 32u - args.w;
                const double two_w = double(uint64_t(1) << args.w);
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    const uint32_t x1a = a1[j] >> shift, x2a = a2[j] >> shift;
                    const uint32_t x1b = b1[j] >> shift, x2b = b2[j] >> shift;
                    const bool oka = x1a != args.a0 && x1a != args.a;
                    const bool okb = x1b != args.a0 && x1b != args.a;
                    v[2 * j] = prngd_map<FAM>(x1a, x2a, args, two_w);
                    v[2 * j + 1] = prngd_map<FAM>(x1b, x2b, args, two_w);
                    acc |= (uint32_t(oka) << (2 * j)) | (uint32_t(okb) << (2 * j + 1));
                }
            }
        } else if (fam_base(FAM) == FAM_PHILOX32) {
            // x in [0, 2^32 - 1]: keep x1 unless x1 + 1 wraps to 0 or is 1
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const uint64_t blk = blk0 + uint32_t(j) * B + tid;
                const Words4 r = philox4x32_10(uint32_t(blk), uint32_t(blk >> 32), 0u,
                                               seg.stream_id, k0, k1);
                const bool oka = r.v0 + 1u >= 2u;
                const bool okb = r.v2 + 1u >= 2u;
                v[2 * j] = map_hi_lo<FAM>(r.v0 - 1u, r.v1, 4294967296.0, args);
                v[2 * j + 1] = map_hi_lo<FAM>(r.v2 - 1u, r.v3, 4294967296.0, args);
                acc |= (uint32_t(oka) << (2 * j)) | (uint32_t(okb) << (2 * j + 1));
            }
        } else {
            const uint32_t shift = 32u - args.w;
            const double two_w = double(uint64_t(1) << args.w);
#pragma unroll
            for (int j = 0; j < J; ++j) {
                uint32_t x1a, x2a, x1b, x2b;
                if (fam_base(FAM) == FAM_PHILOX) {
                    const uint64_t blk = blk0 + uint32_t(j) * B + tid;
                    const Words4 r = philox4x32_10(uint32_t(blk), uint32_t(blk >> 32), 0u,
                                                   seg.stream_id, k0, k1);
                    x1a = r.v0 >> shift;
                    x2a = r.v1 >> shift;
                    x1b = r.v2 >> shift;
                    x2b = r.v3 >> shift;
                } else {
                    const uint64_t p = wb + 2u * (uint32_t(j) * B + tid);
                    const uint64_t mask = (uint64_t(1) << args.w) - 1;
                    x1a = uint32_t((p >> args.w) & mask);
                    x2a = uint32_t(p & mask);
                    x1b = uint32_t(((p + 1) >> args.w) & mask);
                    x2b = uint32_t((p + 1) & mask);
                }
                const bool oka = x1a != args.a0 && x1a != args.a;
                const bool okb = x1b != args.a0 && x1b != args.a;
                v[2 * j] = prngd_map<FAM>(x1a, x2a, args, two_w);
                v[2 * j + 1] = prngd_map<FAM>(x1b, x2b, args, two_w);
                acc |= (uint32_t(oka) << (2 * j)) | (uint32_t(okb) << (2 * j + 1));
            }
        }
        if (lo_off != 0) {
            // clipped first window: pairs before the start position are not
            // part of this fill
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const uint32_t q = pair_q(j);
                if (q < lo_off)
                    acc &= ~(1u << (2 * j));
                if (q + 1 < lo_off)
                    acc &= ~(1u << (2 * j + 1));
            }
        }
        clean = !block_any(lo_off != 0 || acc != kAll);
        if (clean)
            return T;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const uint64_t ba = __ballot((acc >> (2 * j)) & 1u);
            const uint64_t bb = __ballot((acc >> (2 * j + 1)) & 1u);
            if (lane == 0)
                s_off[group(j)] = uint32_t(__popcll(ba) + __popcll(bb));
        }
        __syncthreads();
        if (wave == 0)
            wave0_scan<E>(s_off, lane);
        __syncthreads();
        return uniform_u32(s_off[E]);
    }

    // Store the kept outputs of window `wb` at segment offset `excl`.
    __device__ __forceinline__ void store(const LaunchArgs &args, const Segment &seg,
                                          uint64_t wb, uint64_t excl, uint64_t *next_counter,
                                          const uint32_t *s_off)
    {
        const uint32_t tid = threadIdx.x;
        const uint64_t n = seg.n;
        if (clean) {
            // pair q of the window is output excl + q
            double *o = seg.out + excl;
            const bool aligned = args.store_mode != 1 &&
                                 (reinterpret_cast<uintptr_t>(o) & 15u) == 0;
            if (excl + T < n) {
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    const uint32_t q = pair_q(j);
                    if (aligned) {
                        store_two(o + q, v[2 * j], v[2 * j + 1], args.store_mode);
                    } else {
                        // 8 bytes off a 16-byte boundary (after a rejection):
                        // two 8-byte stores measured faster here than 16-byte
                        // stores paired across lanes
                        store_one(o + q, v[2 * j], args.store_mode);
                        store_one(o + q + 1, v[2 * j + 1], args.store_mode);
                    }
                }
            } else {
                // the window holds output n - 1
                const uint64_t left = n - excl;
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    const uint32_t q = pair_q(j);
                    if (aligned && q + 1 < left) {
                        store_two(o + q, v[2 * j], v[2 * j + 1], args.store_mode);
                    } else {
                        if (q < left)
                            store_one(o + q, v[2 * j], args.store_mode);
                        if (q + 1 < left)
                            store_one(o + q + 1, v[2 * j + 1], args.store_mode);
                    }
                    if (q + 1 == left || q + 2 == left)
                        *next_counter = wb + left;
                }
            }
            return;
        }
        const uint32_t lane = tid & 63u;
        const uint64_t lt = lanemask_lt(lane);
        double *out = seg.out;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const bool oka = (acc >> (2 * j)) & 1u;
            const bool okb = (acc >> (2 * j + 1)) & 1u;
            const uint64_t ba = __ballot(oka), bb = __ballot(okb);
            const uint64_t pos_a = excl + s_off[group(j)] +
                                   uint32_t(__popcll(ba & lt) + __popcll(bb & lt));
            const uint64_t pos_b = pos_a + (oka ? 1u : 0u);
            if (oka && okb && pos_b < n && args.store_mode != 1 &&
                ((reinterpret_cast<uintptr_t>(out + pos_a) & 15u) == 0)) {
                store_two(out + pos_a, v[2 * j], v[2 * j + 1], args.store_mode);
            } else {
                if (oka && pos_a < n)
                    store_one(out + pos_a, v[2 * j], args.store_mode);
                if (okb && pos_b < n)
                    store_one(out + pos_b, v[2 * j + 1], args.store_mode);
            }
            const bool last_a = oka && pos_a == n - 1;
            const bool last_b = okb && pos_b == n - 1;
            if (last_a || last_b)
                *next_counter = wb + pair_q(j) + (last_a ? 1u : 2u);
        }
    }
};

// ======================================================================
// Philox / enumerate family, store-as-you-go form for the segment-
// sequential kernel, where a window's output offset `excl` is known before
// the window is generated.  Every pair is mapped and stored at once at
// excl + q as if the window kept all its pairs, so no value stays in a
// register.  A window that turns out not to be clean (a rejection, or a
// clipped start) is redone exactly: counts from the kept-pair bits, a scan,
// then the pairs are generated again and stored at their true ranks.  The
// speculative stores it made land either on positions it rewrites or on
// positions that later windows of the same workgroup own and rewrite
// after a barrier; positions at or past n are never written.
// ======================================================================
template <int NW, int PPL, uint32_t FAM>
struct SpecTile {
    static constexpr int B = 64 * NW;
    static constexpr int J = PPL / 2;
    static constexpr uint32_t T = uint32_t(B) * PPL;
    static constexpr int E = J * NW;
    static constexpr uint32_t kAll = PPL == 32 ? 0xFFFFFFFFu : ((1u << PPL) - 1u);

    // The two pairs of thread slot j, as the Eq. (5) operands
    // hi = x1 - a0 - 1 and lo = x2 - b0.  A pair is kept iff hi < hmax with
    // hmax = a - a0 - 1: x1 = a0 wraps hi to 2^32 - 1 and x1 = a gives
    // hi = hmax, the two rejected values of Section 2.
    struct HiLo {
        uint32_t ha, la, hb, lb;
    };

    __device__ __forceinline__ static HiLo words(const LaunchArgs &args, const Segment &seg,
                                                 uint64_t wb, int j)
    {
        const uint32_t tid = threadIdx.x;
        uint32_t x1a, x2a, x1b, x2b;
        if (fam_base(FAM) == FAM_ENUM) {
            const uint64_t q = wb + 2u * (uint32_t(j) * B + tid);
            const uint64_t mask = (uint64_t(1) << args.w) - 1;
            x1a = uint32_t((q >> args.w) & mask);
            x2a = uint32_t(q & mask);
            x1b = uint32_t(((q + 1) >> args.w) & mask);
            x2b = uint32_t((q + 1) & mask);
        } else {
            const uint64_t blk = (wb >> 1) + uint32_t(j) * B + tid;
            const uint32_t k0 = uint32_t(seg.seed), k1 = uint32_t(seg.seed >> 32);
            Words4 r;
            if (wb & 1u) {
                // the window starts on a block's second pair: this thread's
                // pairs are its block's second and the next block's first,
                // which lane + 1 computes; for lane 63 that is the block
                // opening the next wave's slot, the same for the whole wave
                // (all lanes must be here for the shuffle)
                const uint64_t nb = (wb >> 1) + uint32_t(j) * B + 64u * ((tid >> 6) + 1u);
                Words4 u;
                philox4x32_10_lane_and_uniform(
                    Words4{uint32_t(blk), uint32_t(blk >> 32), 0u, seg.stream_id},
                    Words4{uint32_t(nb), uint32_t(nb >> 32), 0u, seg.stream_id}, k0, k1, &r, &u);
                uint32_t n0 = uint32_t(__shfl_down(int(r.v0), 1u, 64));
                uint32_t n1 = uint32_t(__shfl_down(int(r.v1), 1u, 64));
                if ((tid & 63u) == 63u) {
                    n0 = u.v0;
                    n1 = u.v1;
                }
                r = Words4{r.v2, r.v3, n0, n1};
            } else {
                r = philox4x32_10(uint32_t(blk), uint32_t(blk >> 32), 0u, seg.stream_id, k0, k1);
            }
            if (fam_base(FAM) == FAM_PHILOX32) {
                x1a = r.v0; x2a = r.v1; x1b = r.v2; x2b = r.v3;
            } else {
                const uint32_t shift = 32u - args.w;
                x1a = r.v0 >> shift; x2a = r.v1 >> shift;
                x1b = r.v2 >> shift; x2b = r.v3 >> shift;
            }
        }
        if (fam_base(FAM) == FAM_PHILOX32)
            return {x1a - 1u, x2a, x1b - 1u, x2b};
        return {x1a - args.a0 - 1u, x2a - args.b0, x1b - args.a0 - 1u, x2b - args.b0};
    }

    __device__ __forceinline__ static double two_w(const LaunchArgs &args)
    {
        return fam_base(FAM) == FAM_PHILOX32 ? 4294967296.0 : double(uint64_t(1) << args.w);
    }

    __device__ __forceinline__ static uint32_t hmax(const LaunchArgs &args)
    {
        return fam_base(FAM) == FAM_PHILOX32 ? 0xFFFFFFFEu : args.a - args.a0 - 1u;
    }

    // Accepted pairs of window `wb` from window offset lo_off on, without
    // storing anything.
    __device__ __forceinline__ static uint32_t count_kept(const LaunchArgs &args,
                                                          const Segment &seg, uint64_t wb,
                                                          uint32_t lo_off, uint32_t *s_off)
    {
        const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
        const uint32_t hm = hmax(args);
        uint32_t rej = 0;
#pragma unroll 2
        for (int j = 0; j < J; ++j) {
            const uint32_t q = 2u * (uint32_t(j) * B + tid);
            const HiLo p = words(args, seg, wb, j);
            rej += uint32_t(p.ha >= hm && q >= lo_off) + uint32_t(p.hb >= hm && q + 1 >= lo_off);
        }
        uint32_t kept = T - lo_off;
        if (block_any(rej != 0)) {
            const uint32_t r = wave_incl_scan(rej, lane);
            if (lane == 63)
                s_off[wave] = r;
            __syncthreads();
            uint32_t total = 0;
#pragma unroll
            for (int k = 0; k < NW; ++k)
                total += s_off[k];
            kept -= uniform_u32(total);
            __syncthreads();
        }
        return kept;
    }

    // Window `wb` produced exactly (from window offset lo_off on) at segment
    // offset excl, writing nothing but its own outputs; returns its number
    // of accepted pairs.  The words are generated once and kept in
    // registers for the ranks and the stores (4 J registers, so only for
    // up to 8 slots).
    __device__ __forceinline__ uint32_t run_exact(const LaunchArgs &args, const Segment &seg,
                                                  uint64_t wb, uint32_t lo_off, uint64_t excl,
                                                  uint64_t *next_counter, uint32_t *s_off)
    {
        const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
        double *o = seg.out + excl;
        const uint64_t left = seg.n - excl;   // outputs still wanted, >= 1
        const uint32_t hm = hmax(args);
        const double tw = two_w(args);
        HiLo ps[J];
        uint32_t acc = 0;
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const uint32_t q = 2u * (uint32_t(j) * B + tid);
            ps[j] = words(args, seg, wb, j);
            const bool oka = ps[j].ha < hm && q >= lo_off;
            const bool okb = ps[j].hb < hm && q + 1 >= lo_off;
            acc |= (uint32_t(oka) << (2 * j)) | (uint32_t(okb) << (2 * j + 1));
        }
        __syncthreads();                      // earlier readers of s_off are done
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const uint64_t ba = __ballot((acc >> (2 * j)) & 1u);
            const uint64_t bb = __ballot((acc >> (2 * j + 1)) & 1u);
            if (lane == 0)
                s_off[j * NW + wave] = uint32_t(__popcll(ba) + __popcll(bb));
        }
        __syncthreads();
        if (wave == 0)
            wave0_scan<E>(s_off, lane);
        __syncthreads();
        const uint64_t lt = lanemask_lt(lane);
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const bool oka = (acc >> (2 * j)) & 1u;
            const bool okb = (acc >> (2 * j + 1)) & 1u;
            const uint64_t ba = __ballot(oka), bb = __ballot(okb);
            const uint32_t pos_a = s_off[j * NW + wave] +
                                   uint32_t(__popcll(ba & lt) + __popcll(bb & lt));
            const uint32_t pos_b = pos_a + (oka ? 1u : 0u);
            if (oka || okb) {
                const double za = map_hi_lo<FAM>(ps[j].ha, ps[j].la, tw, args);
                const double zb = map_hi_lo<FAM>(ps[j].hb, ps[j].lb, tw, args);
                if (oka && pos_a < left)
                    store_one(o + pos_a, za, args.store_mode);
                if (okb && pos_b < left)
                    store_one(o + pos_b, zb, args.store_mode);
            }
            const uint32_t q = 2u * (uint32_t(j) * B + tid);
            if (oka && pos_a + 1 == left)
                *next_counter = wb + q + 1;
            if (okb && pos_b + 1 == left)
                *next_counter = wb + q + 2;
        }
        const uint32_t total = uniform_u32(s_off[E]);
        __syncthreads();
        return total;
    }

    // Produce window `wb` (from window offset lo_off on) at segment offset
    // excl; returns the window's number of accepted pairs.  With kSpec the
    // pairs are stored as they are generated (a window that turns out not
    // to be clean leaves stale values on up to T positions past its own
    // outputs); without it the window is always produced exactly and
    // writes nothing but its own outputs.
    template <bool kSpec = true>
    __device__ __forceinline__ uint32_t run(const LaunchArgs &args, const Segment &seg,
                                            uint64_t wb, uint32_t lo_off, uint64_t excl,
                                            uint64_t *next_counter, uint32_t *s_off)
    {
        if constexpr (!kSpec && J <= 8)
            return run_exact(args, seg, wb, lo_off, excl, next_counter, s_off);
        const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
        const uint64_t n = seg.n;
        double *o = seg.out + excl;
        const uint64_t left = n - excl;       // outputs still wanted, >= 1
        const bool aligned = args.store_mode != 1 && (reinterpret_cast<uintptr_t>(o) & 15u) == 0;
        // outputs 8 bytes off a 16-byte boundary: lane i stores its first
        // output with the second one of lane i - 1 (lanes 0 and 63 store
        // one output alone), so the stores stay 16 bytes wide
        const bool shifted = args.store_mode != 1 && !aligned;
        const uint32_t hm = hmax(args);
        const double tw = two_w(args);
        uint32_t acc = 0;
        bool dirty;
        if (kSpec && lo_off == 0 && left > T) {
            // a full window that does not hold output n - 1: no bounds, no
            // counter; one running max of hi finds any rejection
            uint32_t mx = 0;
#pragma unroll 2
            for (int j = 0; j < J; ++j) {
                const uint32_t q = 2u * (uint32_t(j) * B + tid);
                const HiLo p = words(args, seg, wb, j);
                mx = max(mx, max(p.ha, p.hb));
                const double za = map_hi_lo<FAM>(p.ha, p.la, tw, args);
                const double zb = map_hi_lo<FAM>(p.hb, p.lb, tw, args);
                if (aligned) {
                    store_two(o + q, za, zb, args.store_mode);
                } else if (shifted) {
                    const double prev = wave_shr1(zb);
                    if (lane == 0)
                        store_one(o + q, za, args.store_mode);
                    else
                        store_two(o + q - 1, prev, za, args.store_mode);
                    if (lane == 63)
                        store_one(o + q + 1, zb, args.store_mode);
                } else {
                    store_one(o + q, za, args.store_mode);
                    store_one(o + q + 1, zb, args.store_mode);
                }
            }
            dirty = block_any(mx >= hm);
            if (!dirty)
                return T;
#pragma unroll 1
            for (int j = 0; j < J; ++j) {
                const HiLo p = words(args, seg, wb, j);
                acc |= (uint32_t(p.ha < hm) << (2 * j)) | (uint32_t(p.hb < hm) << (2 * j + 1));
            }
        } else {
#pragma unroll 2
            for (int j = 0; j < J; ++j) {
                const uint32_t q = 2u * (uint32_t(j) * B + tid);
                const HiLo p = words(args, seg, wb, j);
                const bool oka = p.ha < hm && q >= lo_off;
                const bool okb = p.hb < hm && q + 1 >= lo_off;
                acc |= (uint32_t(oka) << (2 * j)) | (uint32_t(okb) << (2 * j + 1));
                if (kSpec && lo_off == 0) {
                    const double za = map_hi_lo<FAM>(p.ha, p.la, tw, args);
                    const double zb = map_hi_lo<FAM>(p.hb, p.lb, tw, args);
                    if (aligned && q + 1 < left) {
                        store_two(o + q, za, zb, args.store_mode);
                    } else {
                        if (q < left)
                            store_one(o + q, za, args.store_mode);
                        if (q + 1 < left)
                            store_one(o + q + 1, zb, args.store_mode);
                    }
                    if (q + 1 == left || q + 2 == left)
                        *next_counter = wb + left;
                }
            }
            dirty = block_any(!kSpec || lo_off != 0 || acc != kAll);
            if (!dirty)
                return T;
        }
        // not clean: exact ranks, then generate and store again
#pragma unroll 1
        for (int j = 0; j < J; ++j) {
            const uint64_t ba = __ballot((acc >> (2 * j)) & 1u);
            const uint64_t bb = __ballot((acc >> (2 * j + 1)) & 1u);
            if (lane == 0)
                s_off[j * NW + wave] = uint32_t(__popcll(ba) + __popcll(bb));
        }
        __syncthreads();
        if (wave == 0)
            wave0_scan<E>(s_off, lane);
        __syncthreads();
        const uint64_t lt = lanemask_lt(lane);
#pragma unroll 1
        for (int j = 0; j < J; ++j) {
            const bool oka = (acc >> (2 * j)) & 1u;
            const bool okb = (acc >> (2 * j + 1)) & 1u;
            const uint64_t ba = __ballot(oka), bb = __ballot(okb);
            const uint32_t pos_a = s_off[j * NW + wave] +
                                   uint32_t(__popcll(ba & lt) + __popcll(bb & lt));
            const uint32_t pos_b = pos_a + (oka ? 1u : 0u);
            const HiLo p = words(args, seg, wb, j);    // every lane: words() may shuffle
            if (oka || okb) {
                const double za = map_hi_lo<FAM>(p.ha, p.la, tw, args);
                const double zb = map_hi_lo<FAM>(p.hb, p.lb, tw, args);
                if (oka && pos_a < left)
                    store_one(o + pos_a, za, args.store_mode);
                if (okb && pos_b < left)
                    store_one(o + pos_b, zb, args.store_mode);
            }
            const uint32_t q = 2u * (uint32_t(j) * B + tid);
            if (oka && pos_a + 1 == left)
                *next_counter = wb + q + 1;
            if (okb && pos_b + 1 == left)
                *next_counter = wb + q + 2;
        }
        const uint32_t total = uniform_u32(s_off[E]);
        __syncthreads();
        return total;
    }
};

// ======================================================================
// MRG32k3a / mixed family.  MRG32k3a is a recurrence, so each thread takes
// PPL consecutive pairs and steps its own state from a jump-ahead start;
// compacted outputs are staged in LDS and written out by consecutive
// threads so that the stores stay coalesced.
// ======================================================================
template <int PPL, uint32_t FAM>
struct MrgTile {
    static constexpr int B = kMrgBlockThreads;
    static constexpr uint32_t T = uint32_t(B) * PPL;
    static constexpr uint32_t R = fam_base(FAM) == FAM_MRG ? 2u : 1u;   // MRG outputs per pair
    static_assert(PPL % 4 == 0, "Philox blocks must not straddle threads");
    static_assert(16 % PPL == 0, "a thread's outputs must share one LDS pad group");

    static constexpr uint32_t kAll = PPL == 32 ? 0xFFFFFFFFu : ((1u << PPL) - 1u);

    double v[PPL];
    uint32_t acc;          // bit i: pair i of this thread kept
    uint32_t thread_off;   // exclusive offset of this thread inside the window

    // This thread's MRG32k3a state at MRG position R (win T + tid PPL).
    __device__ __forceinline__ static Mrg jump(const LaunchArgs &args, const Segment &seg,
                                               uint64_t win)
    {
        Mrg g;
#pragma unroll
        for (int i = 0; i < 6; ++i)
            g.s[i] = seg.mrg[i];
        uint64_t m = win;
        for (int d = 0; d < kMrgDigits && m != 0; ++d, m >>= 8) {
            const uint32_t digit = uint32_t(m & 255u);
            if (digit)
                g.apply(args.mrg_window + (size_t(d) * 256 + digit) * kMrgMatWords);
        }
        g.apply(args.mrg_thread + size_t(threadIdx.x) * kMrgMatWords);
        return g;
    }

    // Pair i of this thread (window offset tid PPL + i): x1 and x2, with the
    // Philox block of the mixed generator's x1 words held in ph.
    __device__ __forceinline__ static void pair(const Segment &seg, uint64_t win, int i, Mrg &g,
                                                Words4 &ph, uint32_t &x1, uint32_t &x2)
    {
        if (fam_base(FAM) == FAM_MIXED) {
            if ((i & 3) == 0) {
                const uint64_t blk = (win * T + threadIdx.x * PPL + i) >> 2;
                ph = philox4x32_10(uint32_t(blk), uint32_t(blk >> 32), 0u, seg.stream_id,
                                   uint32_t(seg.seed), uint32_t(seg.seed >> 32));
            }
            x1 = (i & 3) == 0 ? ph.v0 : (i & 3) == 1 ? ph.v1 : (i & 3) == 2 ? ph.v2 : ph.v3;
            x2 = g.next();
        } else {
            x1 = g.next();
            x2 = g.next();
        }
    }

    // Generates the window's PPL pairs of this thread, mapped, and returns
    // the window's number of kept pairs.  A pair is kept iff
    // hi = x1 - a0 - 1 < a - a0 - 1 (x1 = a0 wraps hi to 2^32 - 1, x1 = a
    // gives hmax), so one running max of hi over the thread's pairs finds
    // any rejection.  Only a window with a rejection or a clipped start
    // walks its pairs again to mark which are kept.
    __device__ __forceinline__ uint32_t generate(const LaunchArgs &args, const Segment &seg,
                                                 uint64_t win, uint32_t lo_off, uint32_t *s_wave)
    {
        const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
        const double two_w = double(uint64_t(1) << args.w);
        const uint32_t hmax = args.a - args.a0 - 1u;
        const uint32_t q0 = tid * PPL;             // window offset of the first pair
        uint32_t mx = 0;
        if (q0 + PPL > lo_off) {
            Mrg g = jump(args, seg, win);
            Words4 ph = {0, 0, 0, 0};
#pragma unroll
            for (int i = 0; i < PPL; ++i) {
                uint32_t x1, x2;
                pair(seg, win, i, g, ph, x1, x2);
                const uint32_t hi = x1 - args.a0 - 1u;
                mx = max(mx, hi);
                v[i] = map_hi_lo<FAM>(hi, x2 - args.b0, two_w, args);
            }
        }
        acc = kAll;
        if (!block_any(mx >= hmax || q0 < lo_off)) {
            thread_off = q0;
            return T;
        }
        {
            acc = 0;
            if (q0 + PPL > lo_off) {
                Mrg g = jump(args, seg, win);
                Words4 ph = {0, 0, 0, 0};
#pragma unroll 1
                for (int i = 0; i < PPL; ++i) {
                    uint32_t x1, x2;
                    pair(seg, win, i, g, ph, x1, x2);
                    const bool ok = q0 + i >= lo_off && x1 - args.a0 - 1u < hmax;
                    acc |= uint32_t(ok) << i;
                }
            }
        }
        const uint32_t c = uint32_t(__popc(acc));
        const uint32_t inc = wave_incl_scan(c, lane);
        if (lane == 63)
            s_wave[wave] = inc;
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int k = 0; k < B / 64; ++k) {
            const uint32_t t = s_wave[k];
            before += uint32_t(k) < wave ? t : 0u;
            total += t;
        }
        thread_off = before + inc - c;
        __syncthreads();       // s_wave is reused by the next window
        return uniform_u32(total);
    }

    __device__ __forceinline__ void store(const LaunchArgs &args, const Segment &seg,
                                          uint64_t win, uint64_t excl, uint32_t total,
                                          uint64_t *next_counter, double *s_vals)
    {
        const uint32_t tid = threadIdx.x;
        const uint64_t n = seg.n;
        if (total == T) {
            // every pair kept: this thread's outputs are window outputs
            // tid PPL .. tid PPL + PPL - 1, one padded LDS run (PPL divides 16)
            double *s = s_vals + pad_index(tid * PPL);
#pragma unroll
            for (int i = 0; i < PPL; ++i)
                s[i] = v[i];
            if (excl < n && n - excl <= T) {
                const uint32_t m = uint32_t(n - 1 - excl);   // window output n - 1
                if (m / PPL == tid)
                    *next_counter = win * T + m + 1;
            }
        } else {
            uint32_t k = thread_off;
#pragma unroll
            for (int i = 0; i < PPL; ++i) {
                if ((acc >> i) & 1u) {
                    s_vals[pad_index(k)] = v[i];
                    if (excl + k == n - 1)
                        *next_counter = win * T + tid * PPL + i + 1;
                    ++k;
                }
            }
        }
        __syncthreads();
        store_staged<B>(seg.out, excl, total, n, s_vals, args.store_mode);
        __syncthreads();       // s_vals is reused by the next window
    }
};

// ======================================================================
// The look-back fill loop shared by both families: tiles in ticket order,
// each tile's offset from the decoupled look-back over its segment.
// ======================================================================
template <class Tile, class Scratch>
__device__ __forceinline__ void lookback_loop(const LaunchArgs &args, Scratch &sh)
{
    constexpr uint32_t T = Tile::T;
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const LaunchState st = read_launch_state(args, &sh.state);
    if (tid == 0)
        sh.next = finish_ticket(args, st, issue_ticket(args));
    __syncthreads();
    for (;;) {
        const uint32_t ticket = __builtin_amdgcn_readfirstlane(sh.next);
        if (ticket == ~0u)
            break;
        uint64_t pending = 0;
        if (tid == 0)
            pending = issue_ticket(args);              // completes during this tile
        Segment seg;
        uint32_t t;
        lookup(args, ticket, &seg, &t);
        const uint32_t par = seg.parity ^ st.flip;
        const uint64_t c0 = load_start(seg, par);
        uint64_t *next_counter = seg.counter + (par ^ 1u);
        const uint64_t w0 = c0 / T;
        const uint64_t win = w0 + t;
        const uint32_t lo_off = t == 0 ? uint32_t(c0 - w0 * T) : 0u;
        Tile tile;
        const uint32_t agg = sh.generate(tile, args, seg, win, lo_off);
        if (t == 0) {
            if (tid == 0) {
                publish(args.status, ticket, pack_status(st.epoch, kFlagPrefix, agg));
                sh.excl = 0;
            }
        } else {
            if (tid == 0)
                publish(args.status, ticket, pack_status(st.epoch, kFlagAggregate, agg));
            if (tid < 64) {
                const uint64_t excl =
                    look_back(args.status, ticket, t, st.epoch, args.ctl, args.error, lane,
                              args.spin_limit ? args.spin_limit : kSpinLimit);
                if (tid == 0) {
                    publish(args.status, ticket, pack_status(st.epoch, kFlagPrefix, excl + agg));
                    sh.excl = excl;
                }
            }
        }
        __syncthreads();
        uint64_t running = sh.excl;
        // a planned tile may lie wholly past output n - 1 (its segment's
        // rejections fell short of the plan): it stores nothing
        if (running < seg.n)
            sh.store(tile, args, seg, win, running, agg, next_counter);
        running += agg;
        // the last tile takes every further window until n outputs
        for (uint64_t w2 = win + 1; t == seg.ntiles - 1 && running < seg.n; ++w2) {
            __syncthreads();
            const uint32_t a2 = sh.generate(tile, args, seg, w2, 0u);
            sh.store(tile, args, seg, w2, running, a2, next_counter);
            running += a2;
        }
        if (tid == 0)
            sh.next = finish_ticket(args, st, pending);
        __syncthreads();
    }
}

// ======================================================================
// The segment-sequential loop: workgroups draw whole segments in ticket
// order and produce each alone, window after window, with an exact
// running offset -- no cross-workgroup waits.  Ticket order keeps the
// segments being written at any moment next to each other in memory.
// The next segment's ticket is drawn while the current one is produced.
// ======================================================================
template <class Tile, class Scratch>
__device__ __forceinline__ void sequential_loop(const LaunchArgs &args, Scratch &sh)
{
    constexpr uint32_t T = Tile::T;
    const uint32_t tid = threadIdx.x;
    const LaunchState st = read_launch_state(args, &sh.state);
    if (tid == 0)
        sh.next = finish_ticket(args, st, issue_ticket(args));
    __syncthreads();
    for (;;) {
        const uint32_t i = __builtin_amdgcn_readfirstlane(sh.next);
        if (i == ~0u)
            break;
        uint64_t pending = 0;
        if (tid == 0)
            pending = issue_ticket(args);
        const Segment seg = load_segment(args.segs, i);
        const uint32_t par = seg.parity ^ st.flip;
        const uint64_t c0 = load_start(seg, par);
        uint64_t *next_counter = seg.counter + (par ^ 1u);
        uint64_t win = c0 / T;
        uint32_t lo_off = uint32_t(c0 - win * T);
        uint64_t running = 0;
        Tile tile;
        while (running < seg.n) {
            const uint32_t agg = sh.generate(tile, args, seg, win, lo_off);
            sh.store(tile, args, seg, win, running, agg, next_counter);
            running += agg;
            ++win;
            lo_off = 0;
            __syncthreads();
        }
        if (tid == 0)
            sh.next = finish_ticket(args, st, pending);
        __syncthreads();
    }
}

// The segment-sequential loop for the store-as-you-go Philox tile.  A
// workgroup never waits for another one here, so it may hold two tickets
// ahead: while segment k is produced, the descriptor of segment k + 1 is
// loaded at once, its start position after the first window, and the
// ticket of segment k + 2 is drawn.  Uniform loads that are in flight
// complete at the latest at the next barrier, after a window of work.
template <int NW, int PPL, uint32_t FAM>
__device__ __forceinline__ void sequential_spec_loop(const LaunchArgs &args, uint32_t *s_off,
                                                     LaunchState *s_state, uint32_t *s_next)
{
    using Tile = SpecTile<NW, PPL, FAM>;
    constexpr uint32_t T = Tile::T;
    const uint32_t tid = threadIdx.x;
    const LaunchState st = read_launch_state(args, s_state);
    if (tid == 0)
        s_next[0] = finish_ticket(args, st, issue_ticket(args));
    __syncthreads();
    uint32_t cur = __builtin_amdgcn_readfirstlane(s_next[0]);
    if (cur == ~0u)
        return;
    if (tid == 0)
        s_next[1] = finish_ticket(args, st, issue_ticket(args));
    Segment seg = load_segment(args.segs, cur);
    uint64_t c0 = load_start(seg, seg.parity ^ st.flip);
    __syncthreads();
    uint32_t nxt = __builtin_amdgcn_readfirstlane(s_next[1]);
    for (;;) {
        uint64_t pending = 0;
        if (tid == 0 && nxt != ~0u)
            pending = issue_ticket(args);            // ticket of the segment after next
        Segment nseg = seg;
        if (nxt != ~0u)
            nseg = load_segment(args.segs, nxt);
        uint64_t nc0 = 0;
        bool nc0_loaded = false;
        const uint32_t par = seg.parity ^ st.flip;
        uint64_t *next_counter = seg.counter + (par ^ 1u);
        uint64_t win = c0 / T;
        uint32_t lo_off = uint32_t(c0 - win * T);
        uint64_t running = 0;
        while (running < seg.n) {
            running += Tile().run(args, seg, win * T, lo_off, running, next_counter, s_off);
            ++win;
            lo_off = 0;
            if (!nc0_loaded && nxt != ~0u) {
                nc0 = load_start(nseg, nseg.parity ^ st.flip);
                nc0_loaded = true;
            }
        }
        if (nxt == ~0u)
            break;
        if (!nc0_loaded)
            nc0 = load_start(nseg, nseg.parity ^ st.flip);
        if (tid == 0)
            s_next[0] = finish_ticket(args, st, pending);
        __syncthreads();
        const uint32_t after = __builtin_amdgcn_readfirstlane(s_next[0]);
        __syncthreads();                              // s_next[0] is rewritten next round
        seg = nseg;
        c0 = nc0;
        cur = nxt;
        nxt = after;
    }
    (void)cur;
}

template <int NW, int PPL, uint32_t FAM>
struct PhiloxScratch {
    using Tile = PhiloxTile<NW, PPL, FAM>;
    uint32_t off[Tile::kOffWords];
    uint64_t excl;
    uint32_t next;
    LaunchState state;

    __device__ __forceinline__ uint32_t generate(Tile &tile, const LaunchArgs &a, const Segment &s,
                                                 uint64_t win, uint32_t lo)
    {
        return tile.generate(a, s, win * Tile::T, lo, off);
    }
    __device__ __forceinline__ void store(Tile &tile, const LaunchArgs &a, const Segment &s,
                                          uint64_t win, uint64_t excl, uint32_t, uint64_t *nc)
    {
        tile.store(a, s, win * Tile::T, excl, nc, off);
    }
};

template <int PPL, uint32_t FAM>
struct MrgScratch {
    using Tile = MrgTile<PPL, FAM>;
    double vals[Tile::T + Tile::T / 16];
    uint32_t wave[kMrgBlockThreads / 64];
    uint64_t excl;
    uint32_t next;
    LaunchState state;

    __device__ __forceinline__ uint32_t generate(Tile &tile, const LaunchArgs &a, const Segment &s,
                                                 uint64_t win, uint32_t lo)
    {
        return tile.generate(a, s, win, lo, wave);
    }
    __device__ __forceinline__ void store(Tile &tile, const LaunchArgs &a, const Segment &s,
                                          uint64_t win, uint64_t excl, uint32_t total, uint64_t *nc)
    {
        tile.store(a, s, win, excl, total, nc, vals);
    }
};

// ======================================================================
// Three words per output (the paper's Conclusion: more than two PRNs
// combined), the two-word method applied twice.  Triple t of a stream is
// words 3t, 3t + 1, 3t + 2; it is kept iff neither x1 nor x2 is a0 or a
// (Section 2's rule for the inner pair (x2, x3), then for the outer pair
// (x1, y = x2 + k x3), whose span is below one step of x1), and maps to
//   N3 = (x1 - a0 - 1) 2^2w + (x2 - a0 - 1) 2^w + (x3 - a0),
//   z' = RN(RN(N3) * S3),  S3 = RN((1 - 2^-3w) / D3),  forced below 1,
// with RN(N3) the correctly rounded value of the exact integer.  Four
// triples are three Philox blocks, so thread (j, tid) of a window starting
// at triple wb (a multiple of 4) takes group g = wb / 4 + j B + tid:
// blocks 3g .. 3g + 2, triples 4g .. 4g + 3 (window offsets
// 4 (j B + tid) + i), and a wave's outputs for one j are contiguous.
// ======================================================================

// RN(U) for U = hi 2^64 + lo < 2^96, round half to even: with hi = 0 one
// fused multiply-add of its 32-bit halves; otherwise the 53 leading bits,
// the next bit and a sticky bit of the rest, from U shifted so that its
// leading one sits at bit 95.
__device__ __forceinline__ double rn_u96(uint32_t hi, uint64_t lo)
{
    if (hi == 0)
        return __builtin_fma(double(uint32_t(lo >> 32)), 4294967296.0, double(uint32_t(lo)));
    const uint32_t lz = uint32_t(__builtin_clz(hi));                 // 0 .. 31
    const uint64_t top = (uint64_t(hi) << (32 + lz)) | (lo >> (32 - lz));
    const uint32_t rest = uint32_t(lo << lz);
    uint64_t m = top >> 11;                                          // 53 bits
    const bool round = (top >> 10) & 1u;
    const bool sticky = (top & 0x3FFu) != 0 || rest != 0;
    if (round && (sticky || (m & 1u)))
        ++m;                                                         // 2^53 at most: exact
    return __builtin_ldexp(double(m), 43 - int(lz));
}

// z' of one kept triple; w < 32 unless the family is FAM_PHILOX32.
template <uint32_t FAM>
__device__ __forceinline__ double map3(uint32_t x1, uint32_t x2, uint32_t x3, const LaunchArgs &a)
{
    const uint32_t w = fam_base(FAM) == FAM_PHILOX32 ? 32u : a.w;
    const uint32_t hi = x1 - a.a0 - 1u;
    const uint64_t M = (uint64_t(x2 - a.a0 - 1u) << w) + (x3 - a.a0);    // Y - Y0 < 2^2w
    double N;
    if (2u * w <= 53u) {
        // M is exact in FP64; the fma rounds the exact sum once
        N = __builtin_fma(double(hi), __builtin_ldexp(1.0, int(2u * w)), double(M));
    } else {
        // U = hi 2^2w + M, 2w >= 54: bits 64 and up, and the low 64 bits
        const uint32_t u2 = 2u * w == 64u ? hi : uint32_t(uint64_t(hi) >> (64u - 2u * w));
        const uint64_t u = 2u * w == 64u ? M : (uint64_t(hi) << (2u * w)) | M;
        N = rn_u96(u2, u);
    }
    const double z = N * a.S;
    return z < kBelowOne ? z : kBelowOne;
}

template <int NW, int G, uint32_t FAM>
struct TripleTile {
    static constexpr int B = 64 * NW;
    static constexpr int PPL = 4 * G;                 // triples per thread
    static constexpr uint32_t T = uint32_t(B) * PPL;  // triples per window
    static constexpr int E = G * NW;                  // (j, wave) groups in triple order
    static constexpr int kOffWords = E + 1;
    static constexpr uint32_t kAll = PPL == 32 ? 0xFFFFFFFFu : ((1u << PPL) - 1u);

    double v[PPL];
    uint32_t acc;          // bit 4j + i: triple i of slot j kept
    bool clean;            // every triple of the window kept

    // The 12 words of group g: triple 4g + i is (x[3i], x[3i + 1], x[3i + 2]).
    __device__ __forceinline__ static void group_words(const LaunchArgs &args,
                                                       const Segment &seg, uint64_t g,
                                                       uint32_t x[12])
    {
        if (fam_base(FAM) == FAM_ENUM) {
            const uint64_t mask = (uint64_t(1) << args.w) - 1;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint64_t t = 4 * g + uint32_t(i);
                x[3 * i] = uint32_t((t >> (2 * args.w)) & mask);
                x[3 * i + 1] = uint32_t((t >> args.w) & mask);
                x[3 * i + 2] = uint32_t(t & mask);
            }
        } else {
            const uint32_t sh = fam_base(FAM) == FAM_PHILOX32 ? 0u : 32u - args.w;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const uint64_t blk = 3 * g + uint32_t(b);
                const Words4 r = philox4x32_10(uint32_t(blk), uint32_t(blk >> 32), 0u,
                                               seg.stream_id, uint32_t(seg.seed),
                                               uint32_t(seg.seed >> 32));
                x[4 * b] = r.v0 >> sh;
                x[4 * b + 1] = r.v1 >> sh;
                x[4 * b + 2] = r.v2 >> sh;
                x[4 * b + 3] = r.v3 >> sh;
            }
        }
    }

    // Generate the window of T triples from triple wb (a multiple of 4), from
    // window offset lo_off on; returns its number of kept triples, and for
    // a window that is not clean leaves each (j, wave) group's exclusive
    // offset in s_off.
    __device__ __forceinline__ uint32_t generate(const LaunchArgs &args, const Segment &seg,
                                                 uint64_t wb, uint32_t lo_off, uint32_t *s_off)
    {
        const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
        const uint32_t hmax = args.a - args.a0 - 1u;
        acc = 0;
#pragma unroll
        for (int j = 0; j < G; ++j) {
            uint32_t x[12];
            group_words(args, seg, (wb >> 2) + uint32_t(j) * B + tid, x);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const bool ok = x[3 * i] - args.a0 - 1u < hmax &&
                                x[3 * i + 1] - args.a0 - 1u < hmax;
                v[4 * j + i] = map3<FAM>(x[3 * i], x[3 * i + 1], x[3 * i + 2], args);
                acc |= uint32_t(ok) << (4 * j + i);
            }
        }
        if (lo_off != 0) {
#pragma unroll
            for (int j = 0; j < G; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (4u * (uint32_t(j) * B + tid) + uint32_t(i) < lo_off)
                        acc &= ~(1u << (4 * j + i));
        }
        clean = !block_any(lo_off != 0 || acc != kAll);
        if (clean)
            return T;
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const uint32_t c = uint32_t(__popc((acc >> (4 * j)) & 15u));
            const uint32_t inc = wave_incl_scan(c, lane);
            if (lane == 63)
                s_off[j * NW + wave] = inc;
        }
        __syncthreads();
        if (wave == 0)
            wave0_scan<E>(s_off, lane);
        __syncthreads();
        return uniform_u32(s_off[E]);
    }

    // Store the kept outputs of window wb at segment offset excl.
    __device__ __forceinline__ void store(const LaunchArgs &args, const Segment &seg,
                                          uint64_t wb, uint64_t excl, uint64_t *next_counter,
                                          const uint32_t *s_off)
    {
        const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
        const uint64_t n = seg.n;
        if (clean) {
            // triple q of the window is output excl + q
            double *o = seg.out + excl;
            const bool aligned = args.store_mode != 1 &&
                                 (reinterpret_cast<uintptr_t>(o) & 15u) == 0;
            const bool past = excl + T < n;    // the window does not hold output n - 1
            const uint64_t left = n - excl;
#pragma unroll
            for (int j = 0; j < G; ++j) {
                const uint32_t q = 4u * (uint32_t(j) * B + tid);
                if (aligned && (past || q + 3 < left)) {
                    store_two(o + q, v[4 * j], v[4 * j + 1], args.store_mode);
                    store_two(o + q + 2, v[4 * j + 2], v[4 * j + 3], args.store_mode);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (past || q + i < left)
                            store_one(o + q + i, v[4 * j + i], args.store_mode);
                }
                if (!past && q < left && left <= q + 4)
                    *next_counter = wb + left;
            }
            return;
        }
        const uint64_t lt = lanemask_lt(lane);
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const uint32_t bits = (acc >> (4 * j)) & 15u;
            // exclusive rank of this thread's first kept triple in its (j, wave) group
            const uint32_t c = uint32_t(__popc(bits));
            const uint32_t before = wave_incl_scan(c, lane) - c;
            uint64_t pos = excl + s_off[j * NW + wave] + before;
            const uint32_t q = 4u * (uint32_t(j) * B + tid);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if ((bits >> i) & 1u) {
                    if (pos < n)
                        store_one(seg.out + pos, v[4 * j + i], args.store_mode);
                    if (pos == n - 1)
                        *next_counter = wb + q + uint32_t(i) + 1;
                    ++pos;
                }
            }
        }
        (void)lt;
    }
};

template <int NW, int G, uint32_t FAM>
struct TripleScratch {
    using Tile = TripleTile<NW, G, FAM>;
    uint32_t off[Tile::kOffWords];
    uint64_t excl;
    uint32_t next;
    LaunchState state;

    __device__ __forceinline__ uint32_t generate(Tile &tile, const LaunchArgs &a, const Segment &s,
                                                 uint64_t win, uint32_t lo)
    {
        return tile.generate(a, s, win * Tile::T, lo, off);
    }
    __device__ __forceinline__ void store(Tile &tile, const LaunchArgs &a, const Segment &s,
                                          uint64_t win, uint64_t excl, uint32_t, uint64_t *nc)
    {
        tile.store(a, s, win * Tile::T, excl, nc, off);
    }
};

template <int NW, int G, uint32_t FAM>
__global__ __launch_bounds__(64 * NW) void fill_triple_kernel(LaunchArgs args)
{
    __shared__ TripleScratch<NW, G, FAM> sh;
    lookback_loop<TripleTile<NW, G, FAM>>(args, sh);
}

template <int NW, int G, uint32_t FAM>
__global__ __launch_bounds__(64 * NW) void seq_triple_kernel(LaunchArgs args)
{
    __shared__ TripleScratch<NW, G, FAM> sh;
    sequential_loop<TripleTile<NW, G, FAM>>(args, sh);
}

template <int NW, int PPL, uint32_t FAM>
__global__ __launch_bounds__(64 * NW) void fill_philox_kernel(LaunchArgs args)
{
    __shared__ PhiloxScratch<NW, PPL, FAM> sh;
    lookback_loop<PhiloxTile<NW, PPL, FAM>>(args, sh);
}

template <int PPL, uint32_t FAM>
__global__ __launch_bounds__(kMrgBlockThreads) void fill_mrg_kernel(LaunchArgs args)
{
    __shared__ MrgScratch<PPL, FAM> sh;
    lookback_loop<MrgTile<PPL, FAM>>(args, sh);
}

template <int NW, int PPL, uint32_t FAM>
__global__ __launch_bounds__(64 * NW) void seq_philox_kernel(LaunchArgs args)
{
    __shared__ uint32_t s_off[SpecTile<NW, PPL, FAM>::E + 1];
    __shared__ LaunchState s_state;
    __shared__ uint32_t s_next[2];
    sequential_spec_loop<NW, PPL, FAM>(args, s_off, &s_state, s_next);
}

// ======================================================================
// Speculative fill for configurations whose rejections are rare (w = 32:
// one pair in 2^31).  One workgroup per tile, no tickets and no waits:
// tile t of a segment assumes that the segment's earlier tiles rejected
// exactly the pairs it has heard of, and stores its window at once at the
// offset that gives.  Tiles whose window rejects pairs append
// (tile, count) to a rejection list, which later tiles read as their
// hint; each tile records the hint it used.  A repair launch that follows
// in stream order recomputes every tile's true offset from the complete
// list and produces again exactly the tiles that (a) assumed too few
// earlier rejections, (b) may hold stale values written there by an
// earlier tile, or (c) hold the segment's last output (so that the next
// pair counter is the true one).  With no rejection in the launch the
// repair launch reads one word and exits.
// ======================================================================
// Start of a speculative tile: its segment, its index t in the segment,
// its segment's start position, and its hint -- the rejections the
// segment's earlier tiles have published so far (read by wave 0,
// broadcast through LDS, recorded for the repair pass).  The list length,
// the replay parity and both halves of the position slot are independent
// loads, issued together; SINGLE launches take the segment from the
// kernel arguments.
struct TileStart {
    Segment seg;
    uint32_t t;
    uint32_t par;
    uint64_t c0;
    uint32_t used;
};

// The hint of tile g: the rejections its segment's earlier tiles have
// published by now (wave 0 reads the list, LDS broadcasts, thread 0
// records it for the repair pass).
__device__ __forceinline__ uint32_t read_hint(const LaunchArgs &args, const TileStart &ts,
                                              uint32_t g, uint32_t *s_hint)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    if (tid < 64) {
        uint32_t used = 0;
        const uint32_t cnt = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&args.spec->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (ts.t > 0 && cnt != 0) {
            const uint32_t lim = cnt < kHintEntries ? cnt : kHintEntries;
            for (uint32_t i = lane; i < lim; i += 64) {
                const uint64_t e = __hip_atomic_load(&args.rejlist[i], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t et = uint32_t(e >> 32);        // tile + 1; 0 = not written yet
                if (et > ts.seg.tile_begin && et <= g)
                    used += uint32_t(e);
            }
            used = wave_incl_scan(used, lane);
        }
        if (lane == 63)
            *s_hint = used;
    }
    __syncthreads();
    const uint32_t used = __builtin_amdgcn_readfirstlane(*s_hint);
    if (tid == 0)
        args.hint[g] = used;
    return used;
}

// A tile's segment, index and start position, without its hint.
template <bool SINGLE>
__device__ __forceinline__ TileStart tile_start(const LaunchArgs &args, uint32_t g)
{
    const uint32_t flip = ((constant_u32 *)args.flip)[0];
    TileStart ts;
    if (SINGLE) {
        ts.seg = args.seg0;
        ts.t = g;
    } else {
        lookup(args, g, &ts.seg, &ts.t);
    }
    const uint64_t c_a = ((constant_u64 *)ts.seg.counter)[0];
    const uint64_t c_b = ((constant_u64 *)ts.seg.counter)[1];
    ts.par = (ts.seg.parity ^ flip) & 1u;
    ts.c0 = ts.par ? c_b : c_a;
    ts.used = 0;
    return ts;
}

template <bool SINGLE>
__device__ __forceinline__ TileStart spec_prologue(const LaunchArgs &args, uint32_t g,
                                                   uint32_t *s_hint)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    uint32_t cnt = 0;
    if (tid < 64)
        cnt = __hip_atomic_load(&args.spec->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t flip = ((constant_u32 *)args.flip)[0];
    TileStart ts;
    if (SINGLE) {
        ts.seg = args.seg0;
        ts.t = g;
    } else {
        lookup(args, g, &ts.seg, &ts.t);
    }
    const uint64_t c_a = ((constant_u64 *)ts.seg.counter)[0];
    const uint64_t c_b = ((constant_u64 *)ts.seg.counter)[1];
    ts.par = (ts.seg.parity ^ flip) & 1u;
    ts.c0 = ts.par ? c_b : c_a;
    if (tid < 64) {
        uint32_t used = 0;
        cnt = __builtin_amdgcn_readfirstlane(cnt);
        if (ts.t > 0 && cnt != 0) {
            const uint32_t lim = cnt < kHintEntries ? cnt : kHintEntries;
            for (uint32_t i = lane; i < lim; i += 64) {
                const uint64_t e = __hip_atomic_load(&args.rejlist[i], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t et = uint32_t(e >> 32);        // tile + 1; 0 = not written yet
                if (et > ts.seg.tile_begin && et <= g)
                    used += uint32_t(e);
            }
            used = wave_incl_scan(used, lane);
        }
        if (lane == 63)
            *s_hint = used;
    }
    __syncthreads();
    ts.used = __builtin_amdgcn_readfirstlane(*s_hint);
    if (tid == 0)
        args.hint[g] = ts.used;
    return ts;
}

// Appends tile g's rejections to the launch's list (thread 0).
__device__ __forceinline__ void publish_rejections(const LaunchArgs &args, uint32_t g,
                                                   uint32_t rej)
{
    if (rej == 0 || threadIdx.x != 0)
        return;
    const uint32_t slot = __hip_atomic_fetch_add(&args.spec->count, 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    if (slot < args.total_tiles)
        __hip_atomic_store(&args.rejlist[slot], (uint64_t(g) + 1u) << 32 | rej,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        __hip_atomic_fetch_or(args.error, kErrSpecList, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_SYSTEM);
}

// Window origin of a Philox-family speculative fill.  The fill's windows
// are the T-pair ranges from pair c0 - lo0 on: tile 0 starts lo0 pairs into
// its window, and tile t >= 1 at pair c0 - lo0 + t T, whose output (before
// rejections) is t T - lo0.  lo0 < 512 is chosen so that those outputs
// start on a 4 KB boundary of the output array (T is a multiple of 512); a
// window then starts on the second pair of a Philox block when c0 - lo0 is
// odd.  A fill that starts before pair lo0 of its stream takes the window
// origin 0 instead (lo0 = c0).  On MI355X stores that straddle 4 KB blocks
// written by different workgroups measured up to 1.2x slower, and 16-byte
// stores one output off the block grid slower still.
template <uint32_t T>
__device__ __forceinline__ uint32_t window_lo0(const Segment &seg, uint64_t c0)
{
    static_assert(T % 512 == 0, "the window must cover whole 4 KB blocks of outputs");
    const uint32_t a = uint32_t((reinterpret_cast<uintptr_t>(seg.out) >> 3) & 511u);
    return c0 >= a ? a : uint32_t(c0);
}

template <int NW, int PPL, uint32_t FAM, bool SINGLE>
__global__ __launch_bounds__(64 * NW) void spec_philox_kernel(LaunchArgs args)
{
    using Tile = SpecTile<NW, PPL, FAM>;
    constexpr uint32_t T = Tile::T;
    __shared__ uint32_t s_off[Tile::E + 1];
    __shared__ uint32_t s_hint;
    const uint32_t g = blockIdx.x;
    const TileStart ts = spec_prologue<SINGLE>(args, g, &s_hint);
    const Segment &seg = ts.seg;
    const uint32_t t = ts.t, used = ts.used;
    const uint64_t c0 = ts.c0;
    uint64_t *next_counter = seg.counter + (ts.par ^ 1u);
    const uint32_t lo0 = window_lo0<T>(seg, c0);
    const uint64_t wb = c0 - lo0 + uint64_t(t) * T;      // the window's first pair
    const uint32_t lo_off = t == 0 ? lo0 : 0u;
    const uint64_t excl = (t == 0 ? 0 : uint64_t(t) * T - lo0) - used;
    uint32_t kept;
    if (excl < seg.n)
        kept = Tile().run(args, seg, wb, lo_off, excl, next_counter, s_off);
    else
        kept = Tile::count_kept(args, seg, wb, lo_off, s_off);
    publish_rejections(args, g, (T - lo_off) - kept);
    // the segment's last tile takes every further window until n outputs
    if (t == seg.ntiles - 1) {
        uint64_t running = excl + kept;
        for (uint64_t w2 = wb + T; running < seg.n; w2 += T)
            running += Tile().run(args, seg, w2, 0u, running, next_counter, s_off);
    }
}

// The speculative fill in its holding form: the tile's window is generated
// into registers first (rejections published at once), and only then is the
// hint read and the window stored at the offset it gives.  A tile thus
// hears of every rejection published while it was generating, which keeps
// the repair pass short where rejections are not rare.  It writes nothing
// but its own outputs.
template <int NW, int PPL, uint32_t FAM, bool SINGLE>
__global__ __launch_bounds__(64 * NW) void spec_hold_kernel(LaunchArgs args)
{
    using Tile = PhiloxTile<NW, PPL, FAM>;
    constexpr uint32_t T = Tile::T;
    __shared__ uint32_t s_off[Tile::kOffWords];
    __shared__ uint32_t s_hint;
    const uint32_t g = blockIdx.x;
    const TileStart ts = tile_start<SINGLE>(args, g);
    const Segment &seg = ts.seg;
    const uint32_t t = ts.t;
    uint64_t *next_counter = seg.counter + (ts.par ^ 1u);
    const uint32_t lo0 = window_lo0<T>(seg, ts.c0);
    const uint64_t wb = ts.c0 - lo0 + uint64_t(t) * T;   // the window's first pair
    const uint32_t lo_off = t == 0 ? lo0 : 0u;
    Tile tile;
    const uint32_t kept = tile.generate(args, seg, wb, lo_off, s_off);
    publish_rejections(args, g, (T - lo_off) - kept);
    const uint32_t used = read_hint(args, ts, g, &s_hint);
    const uint64_t excl = (t == 0 ? 0 : uint64_t(t) * T - lo0) - used;
    if (excl < seg.n)
        tile.store(args, seg, wb, excl, next_counter, s_off);
    if (t == seg.ntiles - 1) {
        uint64_t running = excl + kept;
        for (uint64_t w2 = wb + T; running < seg.n; w2 += T) {
            __syncthreads();
            const uint32_t k2 = tile.generate(args, seg, w2, 0u, s_off);
            tile.store(args, seg, w2, running, next_counter, s_off);
            running += k2;
        }
    }
}

// The speculative fill for MRG32k3a and the mixed generator, in holding
// form: the tile is generated into registers and compacted through LDS as
// in the look-back kernel, its rejections are published, and then it is
// stored at the offset the hint gives.  It writes nothing but its own
// outputs (at a shifted place if the hint was short).
template <int PPL, uint32_t FAM, bool SINGLE>
__global__ __launch_bounds__(kMrgBlockThreads) void spec_mrg_kernel(LaunchArgs args)
{
    using Tile = MrgTile<PPL, FAM>;
    constexpr uint32_t T = Tile::T;
    __shared__ double s_vals[Tile::T + Tile::T / 16];
    __shared__ uint32_t s_wave[kMrgBlockThreads / 64];
    __shared__ uint32_t s_hint;
    const uint32_t g = blockIdx.x;
    const TileStart ts = tile_start<SINGLE>(args, g);
    const Segment &seg = ts.seg;
    const uint32_t t = ts.t;
    uint64_t *next_counter = seg.counter + (ts.par ^ 1u);
    const uint64_t w0 = ts.c0 / T;
    const uint32_t lo0 = uint32_t(ts.c0 - w0 * T);
    const uint64_t win = w0 + t;
    const uint32_t lo_off = t == 0 ? lo0 : 0u;
    Tile tile;
    const uint32_t kept = tile.generate(args, seg, win, lo_off, s_wave);
    publish_rejections(args, g, (T - lo_off) - kept);
    const uint32_t used = read_hint(args, ts, g, &s_hint);
    const uint64_t excl = (t == 0 ? 0 : uint64_t(t) * T - lo0) - used;
    if (excl < seg.n)
        tile.store(args, seg, win, excl, kept, next_counter, s_vals);
    if (t == seg.ntiles - 1) {
        uint64_t running = excl + kept;
        for (uint64_t w2 = win + 1; running < seg.n; ++w2) {
            Tile t2;
            const uint32_t k2 = t2.generate(args, seg, w2, 0u, s_wave);
            t2.store(args, seg, w2, running, k2, next_counter, s_vals);
            running += k2;
        }
    }
}

// What the repair needs to know of one tile of a dirty segment, from the
// complete rejection list: earlier rejections in its segment (P), its own
// rejections, and whether any earlier tile of the segment rejected pairs.
struct TileFacts {
    uint32_t P;
    uint32_t rej;
    bool after_dirty;
};

__device__ __forceinline__ TileFacts tile_facts(const uint64_t *list, uint32_t cnt,
                                                uint32_t tile_begin, uint32_t g)
{
    TileFacts f{0u, 0u, false};
    for (uint32_t i = 0; i < cnt; ++i) {
        const uint64_t e = list[i];
        const uint32_t et = uint32_t(e >> 32);
        if (et > tile_begin && et <= g) {
            f.P += uint32_t(e);
            f.after_dirty = true;
        } else if (et == g + 1) {
            f.rej = uint32_t(e);
        }
    }
    return f;
}

constexpr uint32_t kRepairCache = 1024;    // list entries kept in LDS

// Whether tile g (of segment `seg`, tile index t, whose first tile starts
// lo0 pairs into its window) has to be produced again, and at which true
// offset.
template <uint32_t T>
__device__ __forceinline__ bool needs_redo(const LaunchArgs &args, const uint64_t *list,
                                           uint32_t cnt, const Segment &seg, uint32_t t,
                                           uint32_t lo0, uint32_t g, uint64_t *true_off)
{
    const TileFacts f = tile_facts(list, cnt, seg.tile_begin, g);
    if (!f.after_dirty)
        return false;                 // up to the segment's first dirty tile all is exact
    const uint64_t off = uint64_t(t) * T - lo0 - f.P;    // t >= 1 here
    if (off >= seg.n)
        return false;                 // every output of the tile lies past n
    *true_off = off;
    if (args.hint[g] != f.P)
        return true;                  // (a) assumed too few earlier rejections
    const uint64_t kept = uint64_t(T) - f.rej;
    if (off + kept >= seg.n || t == seg.ntiles - 1)
        return true;                  // (c) holds output n - 1
    // (b) an earlier tile v wrote T positions from its assumed offset,
    // which lies P(v) - hint(v) past its true one, and kept only the first
    // kept(v) of them: stale values reach P(v) - hint(v) + rej(v) past
    // its true end.  Earlier tiles' reach is bounded by P + T.
    uint64_t gap = 0;                 // outputs between v's true end and this tile
    for (uint32_t v = g - 1;; --v) {
        const TileFacts fv = tile_facts(list, cnt, seg.tile_begin, v);
        const uint64_t reach = uint64_t(fv.P - args.hint[v]) + fv.rej;
        if (reach > gap)
            return true;
        if (!fv.after_dirty || v == seg.tile_begin)
            break;                    // v is the first dirty tile or earlier
        const uint32_t tv = v - seg.tile_begin;
        gap += uint64_t(T) - (tv == 0 ? lo0 : 0u) - fv.rej;
        if (gap >= uint64_t(f.P) + T)
            break;
    }
    return false;
}

// How the repair pass produces one tile again, per generator family: the
// tile's first window exactly (nothing written but its own outputs), then,
// for a segment's last tile, every further window until n outputs exist.
template <int NW, int PPL, uint32_t FAM>
struct PhiloxRedo {
    using Tile = SpecTile<NW, PPL, FAM>;
    static constexpr uint32_t T = Tile::T;
    static constexpr uint32_t B = Tile::B;
    struct Scratch {
        uint32_t off[Tile::E + 1];
    };
    // where the fill's windows start (as the speculative kernels chose), and
    // the window argument of tile t: its first pair
    __device__ __forceinline__ static uint32_t lo0(const Segment &seg, uint64_t c0)
    {
        return window_lo0<T>(seg, c0);
    }
    __device__ __forceinline__ static uint64_t window(uint64_t c0, uint32_t lo0, uint32_t t)
    {
        return c0 - lo0 + uint64_t(t) * T;
    }
    __device__ __forceinline__ static void produce(const LaunchArgs &args, const Segment &seg,
                                                   uint64_t wb, uint64_t off, bool last,
                                                   uint64_t *next_counter, Scratch &sh)
    {
        uint64_t running =
            off + Tile().template run<false>(args, seg, wb, 0u, off, next_counter, sh.off);
        if (last)
            for (uint64_t w2 = wb + T; running < seg.n; w2 += T)
                running += Tile().run(args, seg, w2, 0u, running, next_counter, sh.off);
    }
};

template <int PPL, uint32_t FAM>
struct MrgRedo {
    using Tile = MrgTile<PPL, FAM>;
    static constexpr uint32_t T = Tile::T;
    static constexpr uint32_t B = Tile::B;
    struct Scratch {
        double vals[Tile::T + Tile::T / 16];
        uint32_t wave[kMrgBlockThreads / 64];
    };
    // windows on the absolute grid of T pairs; tile t's window index
    __device__ __forceinline__ static uint32_t lo0(const Segment &, uint64_t c0)
    {
        return uint32_t(c0 % T);
    }
    __device__ __forceinline__ static uint64_t window(uint64_t c0, uint32_t, uint32_t t)
    {
        return c0 / T + t;
    }
    __device__ __forceinline__ static void produce(const LaunchArgs &args, const Segment &seg,
                                                   uint64_t win, uint64_t off, bool last,
                                                   uint64_t *next_counter, Scratch &sh)
    {
        uint64_t running = off;
        for (uint64_t w2 = win;; ++w2) {
            Tile tile;
            const uint32_t kept = tile.generate(args, seg, w2, 0u, sh.wave);
            tile.store(args, seg, w2, running, kept, next_counter, sh.vals);
            running += kept;
            if (!last || running >= seg.n)
                break;
        }
    }
};

template <class F>
__global__ __launch_bounds__(F::B) void spec_repair_kernel(LaunchArgs args)
{
    constexpr uint32_t T = F::T;
    constexpr uint32_t B = F::B;
    __shared__ typename F::Scratch sh;
    __shared__ uint64_t s_list[kRepairCache];
    __shared__ uint32_t s_queue[B];
    __shared__ uint64_t s_qoff[B];
    __shared__ uint32_t s_nq;
    const uint32_t tid = threadIdx.x;
    const uint32_t cnt0 =
        __hip_atomic_load(&args.spec->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cnt0 == 0)
        return;
    const uint32_t cnt = cnt0 < args.total_tiles ? cnt0 : args.total_tiles;
    const uint64_t *list = args.rejlist;
    if (cnt <= kRepairCache) {
        for (uint32_t i = tid; i < cnt; i += B)
            s_list[i] = __hip_atomic_load(&args.rejlist[i], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
        list = s_list;
    }
    const uint32_t flip = read_flip(args);
    // pass p: thread tid checks tile (p B + tid) G + blockIdx, so that a run
    // of consecutive tiles to redo is spread over all workgroups
    const uint64_t G = gridDim.x;
    for (uint64_t p = 0; p * B * G + blockIdx.x < args.total_tiles; ++p) {
        if (tid == 0)
            s_nq = 0;
        __syncthreads();
        const uint64_t g64 = (p * B + tid) * G + blockIdx.x;
        if (g64 < args.total_tiles) {
            const uint32_t g = uint32_t(g64);
            Segment seg;
            uint32_t t;
            if (args.segs == nullptr) {
                seg = args.seg0;
                t = g;
            } else {
                seg = args.segs[args.tile_seg[g]];
                t = g - seg.tile_begin;
            }
            const uint64_t c0 = seg.counter[seg.parity ^ flip];
            uint64_t off = 0;
            if (t > 0 && needs_redo<T>(args, list, cnt, seg, t, F::lo0(seg, c0), g, &off)) {
                const uint32_t k = atomicAdd(&s_nq, 1u);
                s_queue[k] = g;
                s_qoff[k] = off;
            }
        }
        __syncthreads();
        const uint32_t nq = s_nq;
        for (uint32_t k = 0; k < nq; ++k) {
            const uint32_t g = __builtin_amdgcn_readfirstlane(s_queue[k]);
            const uint64_t q = s_qoff[k];
            const uint64_t off = uint64_t(__builtin_amdgcn_readfirstlane(uint32_t(q))) |
                                 uint64_t(__builtin_amdgcn_readfirstlane(uint32_t(q >> 32))) << 32;
            Segment seg;
            uint32_t t;
            lookup(args, g, &seg, &t);
            const uint32_t par = seg.parity ^ flip;
            const uint64_t c0 = load_start(seg, par);
            F::produce(args, seg, F::window(c0, F::lo0(seg, c0), t), off, t == seg.ntiles - 1,
                       seg.counter + (par ^ 1u), sh);
        }
        __syncthreads();
    }
    // the last workgroup out clears the list for the next launch
    __shared__ bool s_last;
    __syncthreads();
    if (tid == 0)
        s_last = __hip_atomic_fetch_add(&args.spec->done, 1u, __ATOMIC_ACQ_REL,
                                        __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
    __syncthreads();
    if (s_last) {
        for (uint32_t i = tid; i < cnt; i += B)
            args.rejlist[i] = 0;
        if (tid == 0) {
            __hip_atomic_store(&args.spec->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&args.spec->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int PPL, uint32_t FAM>
__global__ __launch_bounds__(kMrgBlockThreads) void seq_mrg_kernel(LaunchArgs args)
{
    __shared__ MrgScratch<PPL, FAM> sh;
    sequential_loop<MrgTile<PPL, FAM>>(args, sh);
}

// ======================================================================
// Wave-granular speculative fill of a single segment.  A chunk is C = 128
// consecutive pairs, one Philox block per lane; a workgroup of a one-shot
// grid covers 4 CPW consecutive chunks, so workgroups retire in order and
// the region being written at any moment stays narrow.  A chunk knows its
// rejections from one ballot before it stores anything: a clean chunk is
// stored in 16-byte pieces at the offset its hint gives, a chunk with
// rejections ranks its kept pairs by ballot and popcount.  No barrier, no
// LDS.  Each wave reads the rejection list once, at its start; a chunk
// records its hint only when it is nonzero, tagged with the launch epoch.
// ======================================================================
constexpr uint32_t kChunk = kChunkPairs;

// Lanes at or above `first` (0 .. 64) of a wave, as a 64-bit lane mask.
__device__ __forceinline__ uint64_t lanes_from(uint32_t first)
{
    return first >= 64u ? 0ull : ~0ull << first;
}

// a < b for wave-uniform a, b below 2^63, decided on the scalar unit from
// the sign of a - b.  (A 64-bit ordered compare would go to the vector
// unit.)
__device__ __forceinline__ bool uniform_lt(uint64_t a, uint64_t b)
{
    return int32_t(__builtin_amdgcn_readfirstlane(uint32_t((a - b) >> 32))) < 0;
}

// Whether a chunk at wave-uniform offset excl holds 128 outputs below
// n - 1: all its outputs are stored and none of them is the last one
// (whose chunk writes the next position).
__device__ __forceinline__ bool chunk_fits(uint64_t excl, uint64_t n)
{
    return uniform_lt(excl + kChunk, n);
}

template <uint32_t FAM>
struct WaveChunk {
    using HiLo = typename SpecTile<4, 4, FAM>::HiLo;

    // Window `win` of 128 pairs: lane l holds pairs 2l and 2l + 1.  The
    // windows are counted from Philox block blk0 (pair 2 blk0): window w's
    // first block is blk0 + 64 w.  With blk0 = 0 a lane's block index
    // carries nothing into its high word.
    __device__ __forceinline__ static HiLo words(const LaunchArgs &args, const Segment &seg,
                                                 uint64_t win, uint32_t lane, uint64_t blk0 = 0)
    {
        uint32_t x1a, x2a, x1b, x2b;
        if (fam_base(FAM) == FAM_ENUM) {
            const uint64_t q = 2u * blk0 + win * kChunk + 2u * lane;
            const uint64_t mask = (uint64_t(1) << args.w) - 1;
            x1a = uint32_t((q >> args.w) & mask);
            x2a = uint32_t(q & mask);
            x1b = uint32_t(((q + 1) >> args.w) & mask);
            x2b = uint32_t((q + 1) & mask);
        } else {
            const uint64_t blk = blk0 + (win << 6) + lane;
            const uint32_t blk_lo = uint32_t(blk);
            const uint32_t blk_hi = uint32_t(blk >> 32);
            const Words4 r = philox4x32_10(blk_lo, blk_hi, 0u, seg.stream_id,
                                           uint32_t(seg.seed), uint32_t(seg.seed >> 32));
            if (fam_base(FAM) == FAM_PHILOX32) {
                x1a = r.v0; x2a = r.v1; x1b = r.v2; x2b = r.v3;
            } else {
                const uint32_t shift = 32u - args.w;
                x1a = r.v0 >> shift; x2a = r.v1 >> shift;
                x1b = r.v2 >> shift; x2b = r.v3 >> shift;
            }
        }
        if (fam_base(FAM) == FAM_PHILOX32)
            return {x1a - 1u, x2a, x1b - 1u, x2b};
        return {x1a - args.a0 - 1u, x2a - args.b0, x1b - args.a0 - 1u, x2b - args.b0};
    }

    // Produce chunk window `win` (from window offset lo_off on) at segment
    // offset excl (outputs at or past n are dropped); returns the chunk's
    // kept pairs.  Writes nothing but its own outputs.  `full`: the caller
    // knows that lo_off is 0 and that excl + 128 < n, so that a chunk
    // without rejections stores all its outputs with no further test (and
    // holds no last output).
    __device__ __forceinline__ static uint32_t run(const LaunchArgs &args, const Segment &seg,
                                                   uint64_t win, uint32_t lo_off, uint64_t excl,
                                                   uint64_t *next_counter, bool store,
                                                   bool full, uint64_t blk0 = 0)
    {
        const uint32_t lane = threadIdx.x & 63u;
        return emit(args, seg, words(args, seg, win, lane, blk0), 2u * blk0 + win * kChunk,
                    lo_off, excl, next_counter, store, full);
    }

    // The same for a window whose words the caller made: lane l holds
    // pairs 2l and 2l + 1 (x1 - a0 - 1, x2 - b0), the window's first pair
    // is pair0 of the stream.
    __device__ __forceinline__ static uint32_t emit(const LaunchArgs &args, const Segment &seg,
                                                    const HiLo &p, uint64_t pair0,
                                                    uint32_t lo_off, uint64_t excl,
                                                    uint64_t *next_counter, bool store,
                                                    bool full)
    {
        const uint32_t lane = threadIdx.x & 63u;
        const uint32_t hm = fam_base(FAM) == FAM_PHILOX32 ? 0xFFFFFFFEu : args.a - args.a0 - 1u;
        const double tw = fam_base(FAM) == FAM_PHILOX32 ? 4294967296.0 : double(uint64_t(1) << args.w);
        // the ballots straight from the compares; pairs below lo_off
        // (2l < lo_off, 2l + 1 < lo_off) are masked out on the scalar unit
        uint64_t ka = __builtin_amdgcn_ballot_w64(p.ha < hm);
        uint64_t kb = __builtin_amdgcn_ballot_w64(p.hb < hm);
        if (lo_off != 0) {
            ka &= lanes_from((lo_off + 1u) >> 1);
            kb &= lanes_from(lo_off >> 1);
        }
        const uint32_t kept = uint32_t(__popcll(ka) + __popcll(kb));
        if (!store)
            return kept;
        const double za = map_hi_lo<FAM>(p.ha, p.la, tw, args);
        const double zb = map_hi_lo<FAM>(p.hb, p.lb, tw, args);
        double *o = seg.out + excl;
        const uint32_t q = 2u * lane;
        if (full && kept == kChunk) {
            if (args.store_mode != 1 && (reinterpret_cast<uintptr_t>(o) & 15u) == 0) {
                store_two(o + q, za, zb, args.store_mode);
            } else if (args.store_mode != 1) {
                const double prev = wave_shr1(zb);
                if (lane == 0)
                    store_one(o + q, za, args.store_mode);
                else
                    store_two(o + q - 1, prev, za, args.store_mode);
                if (lane == 63)
                    store_one(o + q + 1, zb, args.store_mode);
            } else {
                store_one(o + q, za, args.store_mode);
                store_one(o + q + 1, zb, args.store_mode);
            }
            return kept;
        }
        const bool oka = (ka >> lane) & 1u;
        const bool okb = (kb >> lane) & 1u;
        const uint64_t left = seg.n - excl;            // >= 1
        const uint64_t lt = lanemask_lt(lane);
        const uint32_t pos_a = uint32_t(__popcll(ka & lt) + __popcll(kb & lt));
        const uint32_t pos_b = pos_a + (oka ? 1u : 0u);
        if (oka && pos_a < left)
            store_one(o + pos_a, za, args.store_mode);
        if (okb && pos_b < left)
            store_one(o + pos_b, zb, args.store_mode);
        if (oka && pos_a + 1 == left)
            *next_counter = pair0 + q + 1;
        if (okb && pos_b + 1 == left)
            *next_counter = pair0 + q + 2;
        return kept;
    }
};

__device__ __forceinline__ uint32_t chunk_hint(const LaunchArgs &args, uint32_t g)
{
    const uint64_t r = args.hint64[g];
    return (r >> 24) == args.epoch ? uint32_t(r & 0xFFFFFFu) : 0u;
}

// ======================================================================
// Chunk-speculative fill of a batch (rare rejections): the one-shot grid of
// the chunks of every segment of the batch, one chunk per wave, a chunk
// NWIN consecutive 128-pair windows (one Philox block per lane in each),
// the chunks of one segment consecutive and the segments one after another,
// so the waves in flight write one contiguous stretch of the output arena.
// A prologue kernel writes each segment's record (start chunk, output,
// position slot) for the launch; a wave then needs one scalar load.  Each
// chunk assumes that no earlier chunk of its segment rejected a pair and
// stores at that offset at once; a chunk whose outputs all lie below output
// n - 1 also assumes that it rejects nothing itself and stores each window
// as it is generated (one running maximum finds a rejection afterwards).
// A chunk that rejects marks its segment dirty from its index on; the
// repair kernel then produces every dirty segment again, exactly and in
// order, from its first dirty chunk.  A speculative chunk never writes
// below its true offset (it can only have assumed too few earlier
// rejections) nor past output n - 1, so what a dirty segment's chunks wrote
// lies in the range its repair writes again, and the repair writes the true
// next position last.  A chunk that holds output n - 1 and rejects pairs is
// produced exactly; it marks nothing, since no later chunk holds an output.
// ======================================================================
__device__ __forceinline__ ChunkSeg load_chunk_seg(const ChunkSeg *recs, uint32_t i)
{
    constexpr int kWords = sizeof(ChunkSeg) / 8;
    const constant_u64 *src = (const constant_u64 *)(recs + i);
    uint64_t w[kWords];
#pragma unroll
    for (int k = 0; k < kWords; ++k)
        w[k] = src[k];
    ChunkSeg r;
    __builtin_memcpy(&r, w, sizeof r);
    return r;
}

// The segment of launch-local chunk c: a division by the common chunk count
// (at least 2; multiply-high and shifts), or the chunk -> segment table.
__device__ __forceinline__ uint32_t chunk_segment(const LaunchArgs &args, uint32_t c)
{
    if (args.chunks_per_seg != 0) {
        const uint32_t t = __umulhi(c, args.cps_magic);
        return (t + ((c - t) >> 1)) >> args.cps_shift;
    }
    return ((constant_u32 *)args.tile_seg)[c];
}

__device__ __forceinline__ Segment chunk_segment_view(const ChunkSeg &r)
{
    Segment seg;
    seg.seed = r.seed;
    seg.out = r.out;
    seg.n = r.n;
    seg.stream_id = r.stream_id;
    return seg;
}

template <uint32_t FAM, uint32_t NWIN>
struct BatchChunk {
    static constexpr uint32_t P = NWIN * kChunk;      // pairs per chunk

    // The windows of a clean chunk stored in one of three ways: V = 0
    // 16-byte stores, V = 1 16-byte stores of outputs shifted by one lane
    // (an output arena 8 bytes off a 16-byte boundary), V = 2 8-byte
    // stores.  Returns the running maximum of the windows' hi operands.
    template <int V>
    __device__ __forceinline__ static uint32_t store_windows(const LaunchArgs &args,
                                                             const Segment &seg, uint64_t ch,
                                                             double *o, uint64_t blk0)
    {
        const uint32_t lane = threadIdx.x & 63u;
        const double tw = fam_base(FAM) == FAM_PHILOX32 ? 4294967296.0 : double(uint64_t(1) << args.w);
        const uint32_t mode = args.store_mode;
        const uint32_t q = 2u * lane;
        uint32_t mx = 0;
#pragma unroll
        for (uint32_t j = 0; j < NWIN; ++j) {
            const auto p = WaveChunk<FAM>::words(args, seg, ch * NWIN + j, lane, blk0);
            mx = max(mx, max(p.ha, p.hb));
            const double za = map_hi_lo<FAM>(p.ha, p.la, tw, args);
            const double zb = map_hi_lo<FAM>(p.hb, p.lb, tw, args);
            double *oj = o + j * kChunk;
            if (V == 0) {
                store_two(oj + q, za, zb, mode);
            } else if (V == 1) {
                const double prev = wave_shr1(zb);
                if (lane == 0)
                    store_one(oj + q, za, mode);
                else
                    store_two(oj + q - 1, prev, za, mode);
                if (lane == 63)
                    store_one(oj + q + 1, zb, mode);
            } else {
                store_one(oj + q, za, mode);
                store_one(oj + q + 1, zb, mode);
            }
        }
        return mx;
    }

    // Chunk `ch` (pairs P ch ..) whose P outputs all lie below output
    // n - 1, stored at segment offset excl as if it rejected no pair;
    // returns whether that held.
    __device__ __forceinline__ static bool run_clean(const LaunchArgs &args, const Segment &seg,
                                                     uint64_t ch, uint64_t excl,
                                                     uint64_t blk0 = 0)
    {
        const uint32_t hm = fam_base(FAM) == FAM_PHILOX32 ? 0xFFFFFFFEu : args.a - args.a0 - 1u;
        double *o = seg.out + excl;
        const bool aligned = (reinterpret_cast<uintptr_t>(o) & 15u) == 0;
        uint32_t mx;
        if (args.store_mode != 1 && aligned)
            mx = store_windows<0>(args, seg, ch, o, blk0);
        else if (args.store_mode != 1)
            mx = store_windows<1>(args, seg, ch, o, blk0);
        else
            mx = store_windows<2>(args, seg, ch, o, blk0);
        return __builtin_amdgcn_ballot_w64(mx >= hm) == 0;
    }

    // Chunk `ch` produced exactly from chunk offset lo_off on, at segment
    // offset excl, window by window; returns its accepted pairs.  Windows
    // at or past output n are counted without storing when COUNT_ALL;
    // otherwise the count stops there and P - lo_off is returned (nothing
    // after output n - 1 matters then).
    template <bool COUNT_ALL>
    __device__ __forceinline__ static uint32_t run_exact(const LaunchArgs &args,
                                                         const Segment &seg, uint64_t ch,
                                                         uint32_t lo_off, uint64_t excl,
                                                         uint64_t *next_counter,
                                                         uint64_t blk0 = 0)
    {
        uint64_t running = excl;
        uint32_t kept = 0;
#pragma unroll 1
        for (uint32_t j = lo_off / kChunk; j < NWIN; ++j) {
            const uint32_t lo_j = j == lo_off / kChunk ? lo_off % kChunk : 0u;
            const bool store = uniform_lt(running, seg.n);
            if (!store && !COUNT_ALL)
                return P - lo_off;
            const uint32_t kj =
                WaveChunk<FAM>::run(args, seg, ch * NWIN + j, lo_j, running, next_counter, store,
                                    store && lo_j == 0 && chunk_fits(running, seg.n), blk0);
            running += kj;
            kept += kj;
        }
        return COUNT_ALL || uniform_lt(running, seg.n) ? kept : P - lo_off;
    }

    // Whether a chunk at wave-uniform offset excl holds P outputs below
    // n - 1.
    __device__ __forceinline__ static bool fits(uint64_t excl, uint64_t n)
    {
        return uniform_lt(excl + P, n);
    }
};

// Wave v of the grid takes launch-local chunk v.
template <uint32_t FAM, uint32_t NWIN>
__global__ __launch_bounds__(256) void chunk_batch_kernel(LaunchArgs args)
{
    using C = BatchChunk<FAM, NWIN>;
    constexpr uint32_t P = C::P;
    const uint32_t lane = threadIdx.x & 63u;
    // the wave index is uniform in the wave: say so, so that everything
    // derived from it (chunk, segment, offsets) lives in scalar registers
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t c = blockIdx.x * 4u + wave;
    // Every argument the wave reads, requested at once (one round trip to
    // the scalar cache instead of one per first use), and the segment's
    // record likewise: a wave lives for a few hundred instructions, so its
    // start latency counts.
    {
        const uint32_t total = args.total_tiles, cps = args.chunks_per_seg;
        const uint32_t magic = args.cps_magic, shift = args.cps_shift, mode = args.store_mode;
        const ChunkSeg *recs = args.chunk_segs;
        const uint32_t *tseg = args.tile_seg;
        const double S = args.S;
        asm volatile("" ::"s"(total), "s"(cps), "s"(magic), "s"(shift), "s"(mode), "s"(recs),
                     "s"(tseg), "s"(S));
    }
    if (c >= args.total_tiles)
        return;
    const uint32_t si = chunk_segment(args, c);
    const ChunkSeg r = load_chunk_seg(args.chunk_segs, si);
    asm volatile("" ::"s"(r.seed), "s"(r.out), "s"(r.w0), "s"(r.n), "s"(r.next_counter),
                 "s"(r.stream_id), "s"(r.lo0), "s"(r.tile_begin), "s"(r.ntiles), "s"(r.k_full),
                 "s"(r.k_end));
    const Segment seg = chunk_segment_view(r);
    const uint32_t k = c - r.tile_begin;
    // A chunk past n only matters when an earlier chunk rejected, and then
    // that one marks the segment and the repair produces it.
    if (k >= r.k_end)
        return;
    const uint64_t ch = r.w0 + k;
    const uint32_t lo_off = k == 0 ? r.lo0 : 0u;
    const uint64_t excl = k == 0 ? 0 : uint64_t(k) * P - r.lo0;
    bool clean;
    if (lo_off == 0 && k < r.k_full)
        clean = C::run_clean(args, seg, ch, excl);
    else
        clean = C::template run_exact<false>(args, seg, ch, lo_off, excl, r.next_counter) ==
                P - lo_off;
    if (!clean) {
        if (lane == 0) {
            const uint32_t old = __hip_atomic_fetch_max(&args.first_dirty[si], ~k,
                                                        __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
            if (old == 0u) {
                const uint32_t slot = __hip_atomic_fetch_add(&args.spec->count, 1u,
                                                             __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
                args.dirty_list[slot] = si;    // each segment once: slot < nseg
            }
        }
    } else if (k == r.ntiles - 1) {
        // the segment's last chunk takes every further chunk until n
        // outputs (a dirty segment is left to the repair)
        uint64_t running = excl + (P - lo_off);
        for (uint64_t c2 = ch + 1; uniform_lt(running, r.n); ++c2)
            running += C::template run_exact<false>(args, seg, c2, 0u, running, r.next_counter);
    }
}

// The repair of the chunk form: workgroup b (16 waves) produces dirty
// segments b, b + G, ... again from their first dirty chunk, 16 windows of
// 128 pairs per step: each wave counts its window's accepted pairs, the
// counts meet in LDS (double-buffered, one barrier a step), and each wave
// stores its window at the offset the counts before it give.
constexpr uint32_t kRepairWaves = 16;

template <uint32_t FAM, uint32_t NWIN>
__global__ __launch_bounds__(64 * kRepairWaves) void chunk_repair_kernel(LaunchArgs args)
{
    using C = BatchChunk<FAM, NWIN>;
    __shared__ uint32_t s_kept[2][kRepairWaves];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t cnt = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(&args.spec->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    uint32_t phase = 0;
    for (uint32_t i = blockIdx.x; i < cnt; i += gridDim.x) {
        const uint32_t si = __builtin_amdgcn_readfirstlane(args.dirty_list[i]);
        const uint32_t k0 = ~__builtin_amdgcn_readfirstlane(args.first_dirty[si]);
        const ChunkSeg r = load_chunk_seg(args.chunk_segs, si);
        const Segment seg = chunk_segment_view(r);
        // no chunk before k0 rejected a pair: k0's true offset is the plain
        // one; the first window to produce is the one that holds it
        uint64_t running = k0 == 0 ? 0 : uint64_t(k0) * C::P - r.lo0;
        const uint32_t lo = k0 == 0 ? r.lo0 : 0u;
        uint64_t win = (r.w0 + k0) * NWIN + lo / kChunk;
        uint32_t lo_first = lo % kChunk;
        while (uniform_lt(running, r.n)) {
            const uint64_t w = win + wave;
            const uint32_t lo_w = wave == 0 ? lo_first : 0u;
            const uint32_t kept = WaveChunk<FAM>::run(args, seg, w, lo_w, 0, nullptr, false, false);
            if (lane == 0)
                s_kept[phase][wave] = kept;
            __syncthreads();
            uint32_t before = 0, total = 0;
#pragma unroll
            for (uint32_t v = 0; v < kRepairWaves; ++v) {
                const uint32_t t = s_kept[phase][v];
                before += v < wave ? t : 0u;
                total += t;
            }
            before = uniform_u32(before);
            total = uniform_u32(total);
            const uint64_t off = running + before;
            if (uniform_lt(off, r.n))
                WaveChunk<FAM>::run(args, seg, w, lo_w, off, r.next_counter, true,
                                    lo_w == 0 && chunk_fits(off, r.n));
            running += total;
            win += kRepairWaves;
            lo_first = 0;
            phase ^= 1u;
        }
        if (threadIdx.x == 0)
            args.first_dirty[si] = 0u;
    }
    // the last workgroup out empties the list for the next launch and, in a
    // resident plan, flips the replay parity (the plan's last step)
    __syncthreads();
    if (threadIdx.x == 0 &&
        __hip_atomic_fetch_add(&args.spec->done, 1u, __ATOMIC_ACQ_REL,
                               __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1) {
        __hip_atomic_store(&args.spec->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&args.spec->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (args.toggle)
            *args.toggle ^= 1u;
    }
}

// ======================================================================
// Wave-granular speculative fill of one segment: the one-shot grid of its
// chunks (NWIN windows of 128 pairs), one per wave, counted from the fill's
// start pair rounded down to even (so that an even start puts every chunk
// before the first rejection on a cache line of the output).  A wave reads the
// rejection list once at its start; chunk k stores at the offset that the
// rejections published so far by chunks before it give (its hint,
// recorded when nonzero, tagged with the launch epoch).  A chunk whose
// outputs all lie below output n - 1 stores each window as it is
// generated and checks for rejections afterwards; one that rejected then
// produces itself exactly at the same offset.  Every chunk publishes its
// rejected pairs (chunk + 1, count), also past output n, so that the
// repair pass can compute every chunk's true offset from the complete list.
// ======================================================================
template <uint32_t FAM, uint32_t NWIN>
__global__ __launch_bounds__(256) void spec_wave_kernel(LaunchArgs args)
{
    using C = BatchChunk<FAM, NWIN>;
    constexpr uint32_t P = C::P;
    const uint32_t lane = threadIdx.x & 63u;
    // the wave index is uniform in the wave: say so, so that everything
    // derived from it (chunk, offsets) lives in scalar registers
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t total = args.total_tiles;
    const uint32_t k = blockIdx.x * 4u + wave;
    if (k >= total)
        return;
    // The hint: the first 64 list entries as this wave sees them at its
    // start.  Slots not yet written read 0; the list holds at least 64
    // slots.  The load is issued first so that it overlaps the position
    // loads.
    const uint64_t entry =
        __hip_atomic_load(&args.rejlist[lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const TileStart ts = tile_start<true>(args, 0);
    const Segment &seg = ts.seg;
    uint64_t *next_counter = seg.counter + (ts.par ^ 1u);
    // chunks from the fill's start pair (rounded down to even, so that a
    // lane's pairs are one Philox block): chunk k's outputs start at k P -
    // lo0 less the rejections before it, on a cache line when lo0 = 0
    const uint64_t blk0 = ts.c0 >> 1;
    const uint32_t lo0 = uint32_t(ts.c0 & 1u);
    uint32_t used = 0;
    {
        const uint32_t et = uint32_t(entry >> 32);     // chunk + 1; 0 = none
        const uint32_t mine = et != 0 && et <= k ? uint32_t(entry) : 0u;
        if (__builtin_amdgcn_ballot_w64(mine != 0) != 0) {
            used = mine;
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1)
                used += __shfl_xor(used, d, 64);
            used = __builtin_amdgcn_readfirstlane(used);
            if (lane == 0)
                args.hint64[k] = (args.epoch << 24) | used;
        }
    }
    const uint64_t ch = k;
    const uint32_t lo_off = k == 0 ? lo0 : 0u;
    const uint64_t excl = (k == 0 ? 0 : uint64_t(k) * P - lo0) - used;
    uint32_t kept;
    if (lo_off == 0 && C::fits(excl, seg.n))
        kept = C::run_clean(args, seg, ch, excl, blk0)
                   ? P
                   : C::template run_exact<true>(args, seg, ch, 0u, excl, next_counter, blk0);
    else
        kept = C::template run_exact<true>(args, seg, ch, lo_off, excl, next_counter, blk0);
    const uint32_t rej = (P - lo_off) - kept;
    if (rej != 0 && lane == 0) {
        const uint32_t slot = __hip_atomic_fetch_add(&args.spec->count, 1u, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        if (slot < total)
            __hip_atomic_store(&args.rejlist[slot], (uint64_t(k) + 1u) << 32 | rej,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            __hip_atomic_fetch_or(args.error, kErrSpecList, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_SYSTEM);
    }
    // the last chunk takes every further chunk until n outputs
    if (k == total - 1) {
        uint64_t running = excl + kept;
        for (uint64_t c2 = ch + 1; uniform_lt(running, seg.n); ++c2)
            running += C::template run_exact<false>(args, seg, c2, 0u, running, next_counter,
                                                    blk0);
    }
}

// ======================================================================
// Counted fill of one segment, for streams that reject often enough that
// speculation would redo much of the fill: pass 1 counts every chunk's
// accepted pairs (Philox and the test only, nothing stored), a two-level
// scan turns the counts into exact offsets, and pass 2 produces every chunk
// at its exact offset (a chunk without rejections below output n - 1 in
// 16-byte stores as it is generated, any other one by ranks).  Chunks are
// kCountedWindows windows of 128 pairs on the stream's own grid; chunk 0
// starts lo0 pairs in.  No chunk waits for another and nothing is redone.
// ======================================================================
constexpr uint32_t kCountedWindows = 4;

template <uint32_t FAM>
__global__ __launch_bounds__(256) void counted_count_kernel(LaunchArgs args)
{
    using C = BatchChunk<FAM, kCountedWindows>;
    constexpr uint32_t P = C::P;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t k = blockIdx.x * 4u + wave;
    if (k >= args.total_tiles)
        return;
    const TileStart ts = tile_start<true>(args, 0);
    const Segment &seg = ts.seg;
    const uint64_t w0 = ts.c0 / P;
    const uint32_t lo0 = uint32_t(ts.c0 % P);
    const uint32_t lo_off = k == 0 ? lo0 : 0u;
    uint32_t kept = 0;
#pragma unroll
    for (uint32_t j = 0; j < kCountedWindows; ++j) {
        const uint32_t base = j * kChunk;
        if (lo_off >= base + kChunk)
            continue;
        const uint32_t lo_j = lo_off > base ? lo_off - base : 0u;
        kept += WaveChunk<FAM>::run(args, seg, (w0 + k) * kCountedWindows + j, lo_j, 0,
                                    nullptr, false, false);
    }
    if (lane == 0)
        args.chunk_counts[k] = kept;
}

template <uint32_t FAM>
__global__ __launch_bounds__(256) void counted_produce_kernel(LaunchArgs args)
{
    using C = BatchChunk<FAM, kCountedWindows>;
    constexpr uint32_t P = C::P;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t total = args.total_tiles;
    const uint32_t k = blockIdx.x * 4u + wave;
    if (k >= total)
        return;
    const TileStart ts = tile_start<true>(args, 0);
    const Segment &seg = ts.seg;
    uint64_t *next_counter = seg.counter + (ts.par ^ 1u);
    const uint64_t w0 = ts.c0 / P;
    const uint32_t lo0 = uint32_t(ts.c0 % P);
    const uint64_t off = __builtin_amdgcn_readfirstlane(args.block_offs[k / kScanBlock]) +
                         __builtin_amdgcn_readfirstlane(args.chunk_offs[k]);
    const uint32_t kept = __builtin_amdgcn_readfirstlane(args.chunk_counts[k]);
    const uint64_t ch = w0 + k;
    const uint32_t lo_off = k == 0 ? lo0 : 0u;
    if (uniform_lt(off, seg.n)) {
        if (lo_off == 0 && kept == P && C::fits(off, seg.n))
            (void)C::run_clean(args, seg, ch, off);     // known clean: exact as stored
        else
            (void)C::template run_exact<false>(args, seg, ch, lo_off, off, next_counter);
    }
    // the last chunk takes every further chunk until n outputs
    if (k == total - 1) {
        uint64_t running = off + kept;
        for (uint64_t c2 = ch + 1; uniform_lt(running, seg.n); ++c2)
            running += C::template run_exact<false>(args, seg, c2, 0u, running, next_counter);
    }
}

// Counted fill of one long stream of triples: window k of the fill (T
// triples on the stream's own grid; window 0 from the start position) is
// one workgroup.  Without PRODUCE it counts the window's kept triples; with
// it, after the scan of those counts, it produces the window at its exact
// offset, and the fill's last window continues until n outputs.
template <int NW, int G, uint32_t FAM, bool PRODUCE>
__global__ __launch_bounds__(64 * NW) void counted_triple_kernel(LaunchArgs args)
{
    using Tile = TripleTile<NW, G, FAM>;
    __shared__ uint32_t s_off[Tile::kOffWords];
    const uint32_t k = blockIdx.x;
    const TileStart ts = tile_start<true>(args, 0);
    const Segment &seg = ts.seg;
    const uint64_t w0 = ts.c0 / Tile::T;
    const uint32_t lo0 = uint32_t(ts.c0 % Tile::T);
    Tile tile;
    if (!PRODUCE) {
        const uint32_t kept = tile.generate(args, seg, (w0 + k) * Tile::T, k == 0 ? lo0 : 0u,
                                            s_off);
        if (threadIdx.x == 0)
            args.chunk_counts[k] = kept;
        return;
    }
    uint64_t *next_counter = seg.counter + (ts.par ^ 1u);
    uint64_t excl = __builtin_amdgcn_readfirstlane(args.block_offs[k / kScanBlock]) +
                    __builtin_amdgcn_readfirstlane(args.chunk_offs[k]);
    const bool last = k == args.total_tiles - 1;
    uint32_t lo = k == 0 ? lo0 : 0u;
    for (uint64_t w = w0 + k; uniform_lt(excl, seg.n); ++w, lo = 0u) {
        const uint32_t kept = tile.generate(args, seg, w * Tile::T, lo, s_off);
        tile.store(args, seg, w * Tile::T, excl, next_counter, s_off);
        excl += kept;
        if (!last)
            break;
        __syncthreads();                              // s_off is written again
    }
}

// Whether chunk g (of the single segment) has to be produced again, and
// at which true offset: the rules of needs_redo with chunk hints.
template <uint32_t P>
__device__ __forceinline__ bool chunk_needs_redo(const LaunchArgs &args, const uint64_t *list,
                                                 uint32_t cnt, uint32_t g, uint32_t lo0,
                                                 uint64_t *true_off)
{
    const Segment &seg = args.seg0;
    const TileFacts f = tile_facts(list, cnt, 0u, g);
    if (!f.after_dirty)
        return false;
    const uint64_t off = uint64_t(g) * P - lo0 - f.P;   // g >= 1 here
    if (off >= seg.n)
        return false;
    *true_off = off;
    if (chunk_hint(args, g) != f.P)
        return true;
    if (off + (P - f.rej) >= seg.n || g == args.total_tiles - 1)
        return true;
    uint64_t gap = 0;
    for (uint32_t v = g - 1;; --v) {
        const TileFacts fv = tile_facts(list, cnt, 0u, v);
        const uint64_t reach = uint64_t(fv.P - chunk_hint(args, v)) + fv.rej;
        if (reach > gap)
            return true;
        if (!fv.after_dirty || v == 0)
            break;
        gap += uint64_t(P) - (v == 0 ? lo0 : 0u) - fv.rej;
        if (gap >= uint64_t(f.P) + P)
            break;
    }
    return false;
}

template <uint32_t FAM, uint32_t NWIN>
__global__ __launch_bounds__(256) void spec_wave_repair_kernel(LaunchArgs args)
{
    using C = BatchChunk<FAM, NWIN>;
    constexpr uint32_t P = C::P;
    __shared__ uint64_t s_list[kRepairCache];
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t cnt0 =
        __hip_atomic_load(&args.spec->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cnt0 == 0)
        return;
    const uint32_t total = args.total_tiles;
    const uint32_t cnt = cnt0 < total ? cnt0 : total;
    const uint64_t *list = args.rejlist;
    if (cnt <= kRepairCache) {
        for (uint32_t i = tid; i < cnt; i += 256)
            s_list[i] = __hip_atomic_load(&args.rejlist[i], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
        list = s_list;
    }
    __syncthreads();
    const Segment &seg = args.seg0;
    const uint32_t flip = read_flip(args);
    const uint32_t par = (seg.parity ^ flip) & 1u;
    const uint64_t c0 = load_start(seg, par);
    uint64_t *next_counter = seg.counter + (par ^ 1u);
    const uint64_t blk0 = c0 >> 1;                      // the chunk grid of the fill
    const uint32_t lo0 = uint32_t(c0 & 1u);
    // each wave checks 64 chunks per pass, one per lane, spread over waves
    const uint64_t wid = blockIdx.x * 4u + (tid >> 6);
    const uint64_t W = uint64_t(gridDim.x) * 4u;
    for (uint64_t p = 0; (p * 64) * W + wid < total; ++p) {
        const uint64_t g64 = (p * 64 + lane) * W + wid;
        uint64_t off = 0;
        const bool redo = g64 < total && g64 > 0 &&
                          chunk_needs_redo<P>(args, list, cnt, uint32_t(g64), lo0, &off);
        uint64_t todo = __ballot(redo);
        while (todo) {
            const uint32_t l = uint32_t(__builtin_ctzll(todo));
            todo &= todo - 1;
            const uint32_t g = uint32_t(__shfl(uint32_t(g64), l, 64));
            const uint64_t o = uint64_t(uint32_t(__shfl(uint32_t(off), l, 64))) |
                               uint64_t(uint32_t(__shfl(uint32_t(off >> 32), l, 64))) << 32;
            uint64_t running =
                o + C::template run_exact<false>(args, seg, g, 0u, o, next_counter, blk0);
            if (g == total - 1)
                for (uint64_t c2 = uint64_t(g) + 1; uniform_lt(running, seg.n); ++c2)
                    running += C::template run_exact<false>(args, seg, c2, 0u, running,
                                                            next_counter, blk0);
        }
    }
    __shared__ bool s_last;
    __syncthreads();
    if (tid == 0)
        s_last = __hip_atomic_fetch_add(&args.spec->done, 1u, __ATOMIC_ACQ_REL,
                                        __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
    __syncthreads();
    if (s_last) {
        for (uint32_t i = tid; i < cnt; i += 256)
            args.rejlist[i] = 0;
        if (tid == 0) {
            __hip_atomic_store(&args.spec->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&args.spec->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ======================================================================
// Algorithm 1's single-word consumption (Philox family): a rejected r1
// consumes one word and r2 is the word right after the accepted r1.  The
// pair boundaries then move by one word at every rejected r1, so a segment
// is produced by one workgroup, window by window, carrying the automaton
// state: E (the next word is an r1 candidate) or P (the next word is the
// r2 of the pending r1, the previous window's last word).  A window of
// T = 64 NW 16 consecutive words is generated in registers (4 Philox blocks
// per thread, word q = 4 (j B + tid) + l).  A window with no word equal to
// a0 or a cannot reject: its roles alternate from the incoming state, and
// each thread stores its two outputs per block (pairs (4m, 4m+1),
// (4m+2, 4m+3) from state E; (4m-1, 4m), (4m+1, 4m+2) from state P, the
// word 4m-1 coming from the previous thread), outputs at or past n dropped.
// Any other window -- a candidate rejection, the clipped first window -- is
// walked exactly by wave 0, 64 words at a time, the states before each
// word obtained by a wave scan of the words' transition maps.
// ======================================================================
template <int NW, uint32_t FAM>
struct SingleWords {
    static constexpr int B = 64 * NW;
    static constexpr int J = 4;                     // Philox blocks per thread
    static constexpr uint32_t T = uint32_t(B) * 4u * J;   // words per window

    // the four words of Philox block blk
    __device__ __forceinline__ static void block(const LaunchArgs &args, const Segment &seg,
                                                 uint64_t blk, uint32_t u[4])
    {
        const Words4 r = philox4x32_10(uint32_t(blk), uint32_t(blk >> 32), 0u, seg.stream_id,
                                       uint32_t(seg.seed), uint32_t(seg.seed >> 32));
        const uint32_t sh = fam_base(FAM) == FAM_PHILOX32 ? 0u : 32u - args.w;
        u[0] = r.v0 >> sh;
        u[1] = r.v1 >> sh;
        u[2] = r.v2 >> sh;
        u[3] = r.v3 >> sh;
    }

    // the four words of thread-block (j, tid) of the window starting at word
    // wb: a multiple of 4 for the Philox families, even for the test
    // generator, whose words come two to a pair
    __device__ __forceinline__ static void words(const LaunchArgs &args, const Segment &seg,
                                                 uint64_t wb, int j, uint32_t u[4])
    {
        const uint32_t tid = threadIdx.x;
        if (fam_base(FAM) == FAM_ENUM) {
            const uint64_t mask = (uint64_t(1) << args.w) - 1;
            const uint64_t p0 = (wb >> 1) + 2 * (uint64_t(j) * B + tid), p1 = p0 + 1;
            u[0] = uint32_t((p0 >> args.w) & mask);
            u[1] = uint32_t(p0 & mask);
            u[2] = uint32_t((p1 >> args.w) & mask);
            u[3] = uint32_t(p1 & mask);
        } else {
            block(args, seg, (wb >> 2) + uint32_t(j) * B + tid, u);
        }
    }
};

// Transition map of one word on {E = 0, P = 1}, two bits: bit 0 = image of
// E, bit 1 = image of P.  An accepted r1 candidate moves E to P, a
// rejected one keeps E; an r2 moves P to E.  Words outside the fill: the
// identity (bits 0b10).
__device__ __forceinline__ uint32_t word_map(bool in_fill, bool bad)
{
    return !in_fill ? 0x2u : (bad ? 0x0u : 0x1u);
}

__device__ __forceinline__ uint32_t map_apply(uint32_t m, uint32_t s)
{
    return (m >> s) & 1u;
}

// g after f
__device__ __forceinline__ uint32_t map_then(uint32_t f, uint32_t g)
{
    return map_apply(g, f & 1u) | (map_apply(g, (f >> 1) & 1u) << 1);
}

struct SingleState {
    uint64_t running;     // outputs made so far in the segment
    uint32_t st;          // E = 0, P = 1
    uint32_t pending;     // the accepted r1 when st = P (needed by thread 0 only)
};

template <int NW, uint32_t FAM>
struct SingleScratch {
    static constexpr uint32_t T = SingleWords<NW, FAM>::T;
    union {
        uint32_t words[T];                 // the window's words (exact walk)
        double stage[T / 2 + T / 32];      // a clean window's outputs (staged store)
    };
    uint32_t last[SingleWords<NW, FAM>::J][NW];   // word 3 of lane 63, per (j, wave)
    uint2 head[SingleWords<NW, FAM>::J][NW];      // words 0, 1 of lane 0, per (j, wave)
    uint2 tail;                                   // words 0, 1 of the block after the window
    SingleState state;
};

// MRG32k3a state at output 16 block16 of window `win` (kSingleWindowWords
// outputs per window) of a stream whose base state is seg.mrg: the window
// tables jump by the base-256 digits of the window index, the thread table
// by the 16-output block (tables built for two outputs per pair, 8 pairs
// per thread, 256 threads).
constexpr uint32_t kSingleWindowWords = 4096;

__device__ __forceinline__ Mrg mrg_at_window(const LaunchArgs &args, const Segment &seg,
                                             uint64_t win, uint32_t block16)
{
    Mrg g;
#pragma unroll
    for (int i = 0; i < 6; ++i)
        g.s[i] = seg.mrg[i];
    uint64_t m = win;
    for (int d = 0; d < kMrgDigits && m != 0; ++d, m >>= 8) {
        const uint32_t digit = uint32_t(m & 255u);
        if (digit)
            g.apply(args.mrg_window + (size_t(d) * 256 + digit) * kMrgMatWords);
    }
    g.apply(args.mrg_thread + size_t(block16) * kMrgMatWords);
    return g;
}

// Word q (absolute index) of a single-generator stream.
template <uint32_t FAM>
__device__ __forceinline__ uint32_t single_word_at(const LaunchArgs &args, const Segment &seg,
                                                   uint64_t q)
{
    if (fam_base(FAM) == FAM_MRG) {
        const uint32_t off = uint32_t(q % kSingleWindowWords);
        Mrg g = mrg_at_window(args, seg, q / kSingleWindowWords, off / 16u);
        uint32_t x = 0;
        for (uint32_t k = 0; k <= off % 16u; ++k)
            x = g.next();
        return x;
    }
    if (fam_base(FAM) == FAM_ENUM) {
        const uint64_t mask = (uint64_t(1) << args.w) - 1;
        const uint64_t p = q >> 1;
        return uint32_t((q & 1u) ? (p & mask) : ((p >> args.w) & mask));
    }
    const uint64_t blk = q >> 2;
    const Words4 r = philox4x32_10(uint32_t(blk), uint32_t(blk >> 32), 0u, seg.stream_id,
                                   uint32_t(seg.seed), uint32_t(seg.seed >> 32));
    const uint32_t l = uint32_t(q & 3u);
    const uint32_t v = l == 0 ? r.v0 : l == 1 ? r.v1 : l == 2 ? r.v2 : r.v3;
    return fam_base(FAM) == FAM_PHILOX32 ? v : v >> (32u - args.w);
}

// The words of the window starting at word wb into u (wb even; a multiple of
// T for MRG32k3a, whose jump tables step whole windows); returns whether
// this thread holds a word of the fill (q >= lo) equal to a0 or a.
// MRG32k3a words are stepped 16 consecutive ones per thread from one jump
// and regrouped through LDS.  A Philox window that starts on a block's third
// word gives thread-block (j, tid) words 2 and 3 of its own block and words
// 0 and 1 of the next one, which the next lane holds (lane 63: lane 0 of the
// next wave, through LDS; the window's last thread: one more block).  Every
// thread must call it.
template <int NW, uint32_t FAM>
__device__ __forceinline__ bool single_generate(const LaunchArgs &args, const Segment &seg,
                                                uint64_t wb, uint32_t lo,
                                                uint32_t (&u)[SingleWords<NW, FAM>::J][4],
                                                SingleScratch<NW, FAM> &sm)
{
    using W = SingleWords<NW, FAM>;
    const uint32_t tid = threadIdx.x;
    uint32_t *s_stage = sm.words;
    if (fam_base(FAM) == FAM_MRG) {
        static_assert(fam_base(FAM) != FAM_MRG || (W::T == kSingleWindowWords && W::B == 256),
                      "the MRG32k3a tables assume 256 threads and 4096-word windows");
        Mrg g = mrg_at_window(args, seg, wb / W::T, tid);
        uint32_t x[16];
#pragma unroll
        for (int k = 0; k < 16; ++k)
            x[k] = g.next();
#pragma unroll
        for (int k = 0; k < 16; k += 4)
            *reinterpret_cast<uint4 *>(s_stage + 16u * tid + k) =
                make_uint4(x[k], x[k + 1], x[k + 2], x[k + 3]);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < W::J; ++j) {
            const uint4 v = *reinterpret_cast<const uint4 *>(s_stage + 4u * (uint32_t(j) * W::B + tid));
            u[j][0] = v.x;
            u[j][1] = v.y;
            u[j][2] = v.z;
            u[j][3] = v.w;
        }
    }
    if (fam_base(FAM) != FAM_MRG) {
#pragma unroll
        for (int j = 0; j < W::J; ++j)
            W::words(args, seg, wb, j, u[j]);
    }
    constexpr bool kPhilox = fam_base(FAM) == FAM_PHILOX || fam_base(FAM) == FAM_PHILOX32;
    if (kPhilox && (wb & 2u)) {
        // u[j] holds block (wb >> 2) + j B + tid, the block of the window's
        // first word at j = tid = 0
        const uint32_t lane = tid & 63u, wave = tid >> 6;
        const uint64_t blk0 = wb >> 2;
        if (lane == 0) {
#pragma unroll
            for (int j = 0; j < W::J; ++j)
                sm.head[j][wave] = make_uint2(u[j][0], u[j][1]);
        }
        if (tid == W::B - 1) {
            uint32_t x[4];
            W::block(args, seg, blk0 + uint64_t(W::J) * W::B, x);
            sm.tail = make_uint2(x[0], x[1]);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < W::J; ++j) {
            uint32_t n0 = uint32_t(__shfl_down(int(u[j][0]), 1u, 64));
            uint32_t n1 = uint32_t(__shfl_down(int(u[j][1]), 1u, 64));
            if (lane == 63) {
                const uint2 e = wave + 1 < uint32_t(NW) ? sm.head[j][wave + 1]
                                : j + 1 < W::J          ? sm.head[j + 1][0]
                                                        : sm.tail;
                n0 = e.x;
                n1 = e.y;
            }
            u[j][0] = u[j][2];
            u[j][1] = u[j][3];
            u[j][2] = n0;
            u[j][3] = n1;
        }
    }
    bool bad = false;
#pragma unroll
    for (int j = 0; j < W::J; ++j) {
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const uint32_t q = 4u * (uint32_t(j) * W::B + tid) + l;
            bad |= q >= lo && (u[j][l] == args.a0 || u[j][l] == args.a);
        }
    }
    return bad;
}

// Produces the outputs whose r2 word lies in the window starting at word wb
// (words q >= lo of
// it belong to the fill), from the incoming state ss, which must be the
// same in every thread; stores only outputs below n, and the thread that
// stores output n - 1 writes the next word position.  Leaves ss as the
// state after the window.  `bad` is this thread's flag from
// single_generate.
template <int NW, uint32_t FAM>
__device__ __forceinline__ void single_window_store(const LaunchArgs &args, const Segment &seg,
                                                    uint64_t wb, uint32_t lo,
                                                    const uint32_t (&u)[SingleWords<NW, FAM>::J][4],
                                                    bool bad, SingleState &ss,
                                                    uint64_t *next_counter,
                                                    SingleScratch<NW, FAM> &sm, double two_w)
{
    using W = SingleWords<NW, FAM>;
    constexpr uint32_t T = W::T;
    constexpr int B = W::B, J = W::J;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint64_t n = seg.n;
    const bool exact = block_any(bad) || lo != 0;
    if (ss.running >= n)
        return;
    if (!exact) {
        // outputs 2m and 2m + 1 of the window (m = j B + tid); the window
        // may hold output n - 1 (the r2 word of output k is word 2k + 1 from
        // state E, word 2k from state P)
        double *o = seg.out + ss.running;
        const uint64_t left = n - ss.running;
        const bool aligned = ((reinterpret_cast<uintptr_t>(o) & 15u) == 0);
        const bool whole = left > T / 2;
        const uint32_t r2_of_0 = ss.st == 0 ? 1u : 0u;
        // a whole window not on a 4 KB boundary goes out through LDS
        const bool staged = whole && (reinterpret_cast<uintptr_t>(o) & 4095u) != 0;
        if (ss.st == 0) {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const uint32_t m = uint32_t(j) * B + tid;
                const double za = prngd_map<FAM>(u[j][0], u[j][1], args, two_w);
                const double zb = prngd_map<FAM>(u[j][2], u[j][3], args, two_w);
                if (staged) {
                    sm.stage[pad_index(2 * m)] = za;
                    sm.stage[pad_index(2 * m + 1)] = zb;
                } else if (aligned && (whole || 2 * m + 1 < left)) {
                    store_two(o + 2 * m, za, zb, args.store_mode);
                } else {
                    if (2 * m < left)
                        store_one(o + 2 * m, za, args.store_mode);
                    if (2 * m + 1 < left)
                        store_one(o + 2 * m + 1, zb, args.store_mode);
                }
                if (!whole && (2 * m + 1 == left || 2 * m + 2 == left))
                    *next_counter = wb + 2 * (left - 1) + r2_of_0 + 1;
            }
        } else {
            // word 4m - 1 is word 3 of the previous thread-block
            if (lane == 63) {
#pragma unroll
                for (int j = 0; j < J; ++j)
                    sm.last[j][wave] = u[j][3];
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const uint32_t m = uint32_t(j) * B + tid;
                uint32_t prev = uint32_t(__shfl_up(int(u[j][3]), 1u, 64));
                if (lane == 0) {
                    if (wave > 0)
                        prev = sm.last[j][wave - 1];
                    else if (j > 0)
                        prev = sm.last[j - 1][NW - 1];
                    else
                        prev = ss.pending;
                }
                const double za = prngd_map<FAM>(prev, u[j][0], args, two_w);
                const double zb = prngd_map<FAM>(u[j][1], u[j][2], args, two_w);
                if (staged) {
                    sm.stage[pad_index(2 * m)] = za;
                    sm.stage[pad_index(2 * m + 1)] = zb;
                } else if (aligned && (whole || 2 * m + 1 < left)) {
                    store_two(o + 2 * m, za, zb, args.store_mode);
                } else {
                    if (2 * m < left)
                        store_one(o + 2 * m, za, args.store_mode);
                    if (2 * m + 1 < left)
                        store_one(o + 2 * m + 1, zb, args.store_mode);
                }
                if (!whole && (2 * m + 1 == left || 2 * m + 2 == left))
                    *next_counter = wb + 2 * (left - 1) + r2_of_0 + 1;
            }
            // the window's last word is the next pending r1 (`last` is next
            // written after the barrier that opens the next window's store)
            ss.pending = sm.last[J - 1][NW - 1];
        }
        if (staged) {
            __syncthreads();
            store_staged<B>(seg.out, ss.running, T / 2, n, sm.stage, args.store_mode);
            __syncthreads();   // the stage is reused by the next window
        }
        ss.running += T / 2;
        return;
    }
    // exact walk by wave 0 over the words in order
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
        for (int l = 0; l < 4; ++l)
            sm.words[4u * (uint32_t(j) * B + tid) + l] = u[j][l];
    __syncthreads();
    if (wave == 0) {
        uint32_t state = ss.st, prev_word = ss.pending;
        uint64_t running = ss.running;
        for (uint32_t base = 0; base < T && running < n; base += 64) {
            const uint32_t q = base + lane;
            const uint32_t x = sm.words[q];
            const bool in_fill = q >= lo;
            const bool isbad = x == args.a0 || x == args.a;
            // inclusive scan of the maps, lane order
            uint32_t mp = word_map(in_fill, isbad);
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t other = uint32_t(__shfl_up(int(mp), uint32_t(d), 64));
                if (lane >= uint32_t(d))
                    mp = map_then(other, mp);
            }
            const uint32_t after = map_apply(mp, state);
            uint32_t before = uint32_t(__shfl_up(int(after), 1u, 64));
            if (lane == 0)
                before = state;
            const bool r2 = in_fill && before == 1u;
            uint32_t x1 = uint32_t(__shfl_up(int(x), 1u, 64));
            if (lane == 0)
                x1 = prev_word;
            const uint64_t ball = __ballot(r2);
            const uint64_t pos = running + uint64_t(__popcll(ball & lanemask_lt(lane)));
            if (r2 && pos < n) {
                store_one(seg.out + pos, prngd_map<FAM>(x1, x, args, two_w),
                          args.store_mode == 1 ? 0u : args.store_mode);
                if (pos == n - 1)
                    *next_counter = wb + q + 1;
            }
            running += uint64_t(__popcll(ball));
            state = uint32_t(__shfl(int(after), 63, 64));
            prev_word = uint32_t(__shfl(int(x), 63, 64));
        }
        if (lane == 0) {
            sm.state.running = running;
            sm.state.st = state;
            sm.state.pending = prev_word;
        }
    }
    __syncthreads();
    ss = sm.state;
    __syncthreads();
}

template <int NW, uint32_t FAM>
__global__ __launch_bounds__(64 * NW) void seq_single_kernel(LaunchArgs args)
{
    using W = SingleWords<NW, FAM>;
    constexpr uint32_t T = W::T;
    __shared__ SingleScratch<NW, FAM> sm;
    __shared__ LaunchState s_launch;
    __shared__ uint32_t s_next;
    const uint32_t tid = threadIdx.x;
    const double two_w = fam_base(FAM) == FAM_PHILOX32 ? 4294967296.0 : double(uint64_t(1) << args.w);
    const LaunchState st0 = read_launch_state(args, &s_launch);
    if (tid == 0)
        s_next = finish_ticket(args, st0, issue_ticket(args));
    __syncthreads();
    for (;;) {
        const uint32_t si = __builtin_amdgcn_readfirstlane(s_next);
        if (si == ~0u)
            break;
        uint64_t pending_ticket = 0;
        if (tid == 0)
            pending_ticket = issue_ticket(args);
        const Segment seg = load_segment(args.segs, si);
        const uint32_t par = seg.parity ^ st0.flip;
        const uint64_t c0 = load_start(seg, par);
        uint64_t *next_counter = seg.counter + (par ^ 1u);
        uint64_t wb = (c0 / T) * T;
        uint32_t lo = uint32_t(c0 - wb);
        SingleState ss{0, 0, 0};
        while (ss.running < seg.n) {
            uint32_t u[W::J][4];
            const bool bad = single_generate<NW, FAM>(args, seg, wb, lo, u, sm);
            single_window_store<NW, FAM>(args, seg, wb, lo, u, bad, ss, next_counter, sm, two_w);
            wb += T;
            lo = 0;
        }
        if (tid == 0)
            s_next = finish_ticket(args, st0, pending_ticket);
        __syncthreads();
    }
}

// ======================================================================
// One-word consumption of one long segment across workgroups.  Word r of
// the fill (r = 0 at the start position) is a *candidate* when it equals a0
// or a.  After any candidate the next word is an r1 candidate (a rejected
// r1 keeps state E; an r2, even one equal to a0 or a, returns to E), so the
// i-th candidate is a rejected r1 exactly when r_i - r_{i-1} is odd
// (r_{-1} = -1), and with h the rejected r1 before word r, the state at r is
// E iff r - h is even and floor((r - h) / 2) outputs are complete.  Every
// quantity a window needs thus follows from the candidates before it.
//
// spec_words_kernel: a one-shot grid, tile t = the window of T words that
// starts at word c0 - lo0 + t T.
// The tile generates its words, appends each of its candidates to the
// launch's list ((t + 1) << 32 | word in window), then reads the list and
// takes the rejected r1 among the earlier tiles' candidates it can see (its
// hint h), and produces its window from state (r0 - h) mod 2 at output
// floor((r0 - h) / 2).  Dropping candidates from a set never raises its
// count of rejected r1 (two gaps merge into one whose parity is their sum's),
// so a hint never exceeds the truth and a tile never writes below its true
// offset.  The segment's last tile produces every further window itself.
//
// spec_words_repair_kernel, in stream order: from the complete list it
// computes every tile's true h and produces again the tiles that (a) took a
// smaller h, (b) may hold values a wrong earlier tile wrote past its true
// end (a tile with hint h' < h and c candidates writes at most
// (h - h' + c + 2) / 2 outputs past it), or (c) hold output n - 1, or are the
// last tile, behind a wrong one.  With more candidates than it caches, one
// workgroup produces the segment again from its first dirty window on.
// ======================================================================
__device__ __forceinline__ void publish_word(const LaunchArgs &args, uint32_t t, uint32_t q)
{
    const uint32_t slot =
        __hip_atomic_fetch_add(&args.spec->count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (slot < args.list_cap)
        __hip_atomic_store(&args.rejlist[slot], (uint64_t(t) + 1u) << 32 | q, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    else
        __hip_atomic_fetch_or(args.error, kErrSpecList, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_SYSTEM);
}

// The hint of tile t: rejected r1 among the candidates of tiles before t
// visible in the list now (at most kHintEntries list slots are read).
// Every thread takes part; thread 0 records the hint for the repair pass.
template <uint32_t T>
__device__ __forceinline__ uint32_t read_word_hint(const LaunchArgs &args, uint32_t t, uint32_t lo0,
                                                   int64_t *s_vis, uint32_t *s_nv, uint32_t *s_h)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    if (tid < 64) {
        uint32_t nv = 0;
        const uint32_t cnt = __builtin_amdgcn_readfirstlane(
            __hip_atomic_load(&args.spec->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (t > 0 && cnt != 0) {
            const uint32_t lim = cnt < kHintEntries ? cnt : kHintEntries;
            for (uint32_t base = 0; base < lim; base += 64) {
                const uint32_t i = base + lane;
                uint64_t e = 0;
                if (i < lim)
                    e = __hip_atomic_load(&args.rejlist[i], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t et = uint32_t(e >> 32);        // tile + 1; 0 = not written yet
                const bool vis = et != 0 && et <= t;
                const uint64_t m = __ballot(vis);
                if (vis)
                    s_vis[nv + uint32_t(__popcll(m & lanemask_lt(lane)))] =
                        int64_t(uint64_t(et - 1u) * T + uint32_t(e & 0xFFFFFFFFu)) - int64_t(lo0);
                nv += uint32_t(__popcll(m));
            }
        }
        if (lane == 0) {
            *s_nv = nv;
            *s_h = 0;
        }
    }
    __syncthreads();
    const uint32_t nv = __builtin_amdgcn_readfirstlane(*s_nv);
    if (nv != 0) {
        uint32_t skips = 0;
        for (uint32_t i = tid; i < nv; i += blockDim.x) {
            const int64_t r = s_vis[i];
            int64_t pred = -1;
            for (uint32_t k = 0; k < nv; ++k) {
                const int64_t rk = s_vis[k];
                if (rk < r && rk > pred)
                    pred = rk;
            }
            skips += uint32_t((r - pred) & 1);
        }
        if (skips)
            atomicAdd(s_h, skips);
        __syncthreads();
    }
    const uint32_t h = __builtin_amdgcn_readfirstlane(*s_h);
    if (tid == 0)
        args.hint[t] = h;
    return h;
}

// Incoming state of tile t >= 1 of a fill that starts lo0 words into its
// first window, with h rejected r1 before it.
// Words of a one-word fill's first window that lie before the fill's
// first word c0.  A clean window t >= 1 then starts at output
// floor((t T - lo0) / 2), so lo0 = 2a (c0 even: state E) or 2a - 1 (c0 odd:
// state P, the output taking the word before the window as r1), modulo 1024
// words, puts its outputs on the 4 KB grid of out (a = the 8-byte slot of
// out within its 4 KB block), and every window starts on an even word.
// MRG32k3a keeps windows on multiples of T, the jumps its tables hold.
template <uint32_t FAM, uint32_t T>
__device__ __forceinline__ uint32_t word_lo0(const Segment &seg, uint64_t c0)
{
    static_assert(T % 1024 == 0, "the window must cover whole 4 KB blocks of outputs");
    if (fam_base(FAM) == FAM_MRG)
        return uint32_t(c0 % T);
    const uint32_t a = uint32_t((reinterpret_cast<uintptr_t>(seg.out) >> 3) & 511u);
    const uint32_t lo = (2u * a - (uint32_t(c0) & 1u)) & 1023u;
    return c0 >= lo ? lo : uint32_t(c0 & 1u);
}

template <uint32_t FAM, uint32_t T>
__device__ __forceinline__ SingleState single_entry(const LaunchArgs &args, const Segment &seg,
                                                    uint64_t wb, uint32_t t, uint32_t lo0,
                                                    uint32_t h)
{
    const uint64_t done = uint64_t(t) * T - lo0 - h;   // words used by complete or pending outputs
    SingleState ss;
    ss.running = done >> 1;
    ss.st = uint32_t(done & 1u);
    ss.pending = 0;
    if (ss.st && threadIdx.x == 0)
        ss.pending = single_word_at<FAM>(args, seg, wb - 1u);
    return ss;
}

template <int NW, uint32_t FAM>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(5))) void spec_words_kernel(LaunchArgs args)
{
    using W = SingleWords<NW, FAM>;
    constexpr uint32_t T = W::T;
    constexpr int B = W::B, J = W::J;
    __shared__ SingleScratch<NW, FAM> sm;
    __shared__ int64_t s_vis[kHintEntries];
    __shared__ uint32_t s_nv, s_h;
    const uint32_t tid = threadIdx.x;
    const uint32_t t = blockIdx.x;
    const double two_w = fam_base(FAM) == FAM_PHILOX32 ? 4294967296.0 : double(uint64_t(1) << args.w);
    const TileStart ts = tile_start<true>(args, t);
    const Segment &seg = ts.seg;
    uint64_t *next_counter = seg.counter + (ts.par ^ 1u);
    const uint32_t lo0 = word_lo0<FAM, T>(seg, ts.c0);
    const uint64_t wb = ts.c0 - lo0 + uint64_t(t) * T;   // the window's first word
    const uint32_t lo = t == 0 ? lo0 : 0u;
    uint32_t u[J][4];
    const bool bad = single_generate<NW, FAM>(args, seg, wb, lo, u, sm);
    if (bad) {
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                const uint32_t q = 4u * (uint32_t(j) * B + tid) + l;
                if (q >= lo && (u[j][l] == args.a0 || u[j][l] == args.a))
                    publish_word(args, t, q);
            }
    }
    const uint32_t h = read_word_hint<T>(args, t, lo0, s_vis, &s_nv, &s_h);
    SingleState ss{0, 0, 0};
    if (t > 0)
        ss = single_entry<FAM, T>(args, seg, wb, t, lo0, h);
    single_window_store<NW, FAM>(args, seg, wb, lo, u, bad, ss, next_counter, sm, two_w);
    if (t == seg.ntiles - 1) {
        for (uint64_t w2 = wb + T; ss.running < seg.n; w2 += T) {
            uint32_t v[J][4];
            const bool b2 = single_generate<NW, FAM>(args, seg, w2, 0u, v, sm);
            single_window_store<NW, FAM>(args, seg, w2, 0u, v, b2, ss, next_counter, sm, two_w);
        }
    }
}

// What the repair knows of tile g from the complete candidate list.
struct WordFacts {
    uint32_t h;           // rejected r1 before the tile
    uint32_t c;           // candidates in the tile
    uint32_t k;           // rejected r1 in the tile
    bool after_dirty;     // some earlier tile has a candidate
};

__device__ __forceinline__ WordFacts word_facts(const uint32_t *s_t, const uint8_t *s_skip,
                                                uint32_t cnt, uint32_t g)
{
    WordFacts f{0u, 0u, 0u, false};
    for (uint32_t i = 0; i < cnt; ++i) {
        const uint32_t ti = s_t[i];
        if (ti < g) {
            f.h += s_skip[i];
            f.after_dirty = true;
        } else if (ti == g) {
            f.c += 1u;
            f.k += s_skip[i];
        }
    }
    return f;
}

template <uint32_t T>
__device__ __forceinline__ bool words_need_redo(const LaunchArgs &args, const uint32_t *s_t,
                                                const uint8_t *s_skip, uint32_t cnt,
                                                const Segment &seg, uint32_t lo0, uint32_t g,
                                                uint32_t *true_h)
{
    const WordFacts f = word_facts(s_t, s_skip, cnt, g);
    if (!f.after_dirty)
        return false;                 // up to the first dirty tile all is exact (g >= 1 here)
    const uint64_t r0 = uint64_t(g) * T - lo0;
    const uint64_t off = (r0 - f.h) >> 1;
    if (off >= seg.n)
        return false;                 // every output of the tile lies past n
    *true_h = f.h;
    if (args.hint[g] != f.h)
        return true;                  // (a)
    const uint64_t off_end = (r0 + T - f.h - f.k) >> 1;
    if (off_end >= seg.n || g == seg.ntiles - 1)
        return true;                  // (c)
    // (b) walk back over earlier tiles while their stale writes could reach
    uint64_t gap = 0;
    const uint64_t bound = (uint64_t(cnt) + 2u) / 2u;
    for (uint32_t v = g - 1;; --v) {
        const WordFacts fv = word_facts(s_t, s_skip, cnt, v);
        const uint32_t hv = args.hint[v];
        const uint64_t reach = hv == fv.h ? 0u : (uint64_t(fv.h - hv) + fv.c + 2u) / 2u;
        if (reach > gap)
            return true;
        if (!fv.after_dirty)
            break;                    // v and all before it wrote exactly (v >= 1 past here)
        const uint64_t rv = uint64_t(v) * T - lo0;
        gap += ((rv + T - fv.h - fv.k) >> 1) - ((rv - fv.h) >> 1);
        if (gap >= bound)
            break;
    }
    return false;
}

template <int NW, uint32_t FAM>
__global__ __launch_bounds__(64 * NW) void spec_words_repair_kernel(LaunchArgs args)
{
    using W = SingleWords<NW, FAM>;
    constexpr uint32_t T = W::T;
    constexpr int B = W::B, J = W::J;
    __shared__ SingleScratch<NW, FAM> sm;
    __shared__ int64_t s_r[kRepairCache];
    __shared__ uint32_t s_t[kRepairCache];
    __shared__ uint8_t s_skip[kRepairCache];
    __shared__ uint32_t s_queue[B];
    __shared__ uint32_t s_qh[B];
    __shared__ uint32_t s_nq, s_first;
    __shared__ bool s_last;
    const uint32_t tid = threadIdx.x;
    const uint32_t cnt0 = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(&args.spec->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (cnt0 == 0)
        return;
    const uint32_t cnt = cnt0 < args.list_cap ? cnt0 : args.list_cap;
    const double two_w = fam_base(FAM) == FAM_PHILOX32 ? 4294967296.0 : double(uint64_t(1) << args.w);
    const Segment seg = args.seg0;
    const uint32_t par = (seg.parity ^ read_flip(args)) & 1u;
    const uint64_t c0 = load_start(seg, par);
    uint64_t *next_counter = seg.counter + (par ^ 1u);
    const uint32_t lo0 = word_lo0<FAM, T>(seg, c0);
    const uint64_t wb0 = c0 - lo0;   // the first window's first word
    if (cnt <= kRepairCache) {
        for (uint32_t i = tid; i < cnt; i += B) {
            const uint64_t e = __hip_atomic_load(&args.rejlist[i], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t ti = uint32_t(e >> 32) - 1u;
            s_t[i] = ti;
            s_r[i] = int64_t(uint64_t(ti) * T + uint32_t(e & 0xFFFFFFFFu)) - int64_t(lo0);
        }
        __syncthreads();
        for (uint32_t i = tid; i < cnt; i += B) {
            const int64_t r = s_r[i];
            int64_t pred = -1;
            for (uint32_t k = 0; k < cnt; ++k) {
                const int64_t rk = s_r[k];
                if (rk < r && rk > pred)
                    pred = rk;
            }
            s_skip[i] = uint8_t((r - pred) & 1);
        }
        __syncthreads();
        // pass p: thread tid checks tile (p B + tid) G + blockIdx, so that a
        // run of consecutive tiles to redo is spread over all workgroups
        const uint64_t G = gridDim.x;
        for (uint64_t p = 0; p * B * G + blockIdx.x < seg.ntiles; ++p) {
            if (tid == 0)
                s_nq = 0;
            __syncthreads();
            const uint64_t g64 = (p * B + tid) * G + blockIdx.x;
            uint32_t h = 0;
            if (g64 < seg.ntiles && g64 > 0 &&
                words_need_redo<T>(args, s_t, s_skip, cnt, seg, lo0, uint32_t(g64), &h)) {
                const uint32_t k = atomicAdd(&s_nq, 1u);
                s_queue[k] = uint32_t(g64);
                s_qh[k] = h;
            }
            __syncthreads();
            const uint32_t nq = __builtin_amdgcn_readfirstlane(s_nq);
            for (uint32_t k = 0; k < nq; ++k) {
                const uint32_t g = __builtin_amdgcn_readfirstlane(s_queue[k]);
                const uint32_t hg = __builtin_amdgcn_readfirstlane(s_qh[k]);
                const uint64_t wb = wb0 + uint64_t(g) * T;
                SingleState ss = single_entry<FAM, T>(args, seg, wb, g, lo0, hg);
                uint32_t u[J][4];
                const bool bad = single_generate<NW, FAM>(args, seg, wb, 0u, u, sm);
                single_window_store<NW, FAM>(args, seg, wb, 0u, u, bad, ss, next_counter, sm,
                                             two_w);
                if (g == seg.ntiles - 1) {
                    for (uint64_t w2 = wb + T; ss.running < seg.n; w2 += T) {
                        const bool b2 = single_generate<NW, FAM>(args, seg, w2, 0u, u, sm);
                        single_window_store<NW, FAM>(args, seg, w2, 0u, u, b2, ss, next_counter,
                                                     sm, two_w);
                    }
                }
            }
            __syncthreads();
        }
    } else if (blockIdx.x == 0) {
        // too many candidates to cache: produce the segment again, in
        // order, from the first window that holds one
        if (tid == 0)
            s_first = ~0u;
        __syncthreads();
        uint32_t first = ~0u;
        for (uint32_t i = tid; i < cnt; i += B) {
            const uint64_t e = __hip_atomic_load(&args.rejlist[i], __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t ti = uint32_t(e >> 32) - 1u;
            first = ti < first ? ti : first;
        }
        atomicMin(&s_first, first);
        __syncthreads();
        const uint32_t f = __builtin_amdgcn_readfirstlane(s_first);
        uint64_t wb = wb0 + uint64_t(f) * T;
        uint32_t lo = f == 0 ? lo0 : 0u;
        SingleState ss{0, 0, 0};
        if (f > 0)
            ss = single_entry<FAM, T>(args, seg, wb, f, lo0, 0u);
        while (ss.running < seg.n) {
            uint32_t u[J][4];
            const bool bad = single_generate<NW, FAM>(args, seg, wb, lo, u, sm);
            single_window_store<NW, FAM>(args, seg, wb, lo, u, bad, ss, next_counter, sm, two_w);
            wb += T;
            lo = 0;
        }
    }
    // the last workgroup out clears the list for the next launch
    __syncthreads();
    if (tid == 0)
        s_last = __hip_atomic_fetch_add(&args.spec->done, 1u, __ATOMIC_ACQ_REL,
                                        __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
    __syncthreads();
    if (s_last) {
        for (uint32_t i = tid; i < cnt; i += B)
            args.rejlist[i] = 0;
        if (tid == 0) {
            __hip_atomic_store(&args.spec->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&args.spec->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

}  // namespace
}  // namespace prngd
