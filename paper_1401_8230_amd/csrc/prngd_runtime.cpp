// prngd_runtime.cpp -- host runtime of libprngd: validation, the constants
// of Eq. (5), device state, launch planning, batches, graphs, tuning.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/prngd.h"
#include "prngd_internal.hpp"
#include "prngd_probe.h"

namespace prngd {
const void *fill_kernel_for(uint32_t fam, uint32_t threads, uint32_t ppl, bool seq);
const void *spec_kernel_for(uint32_t fam, uint32_t threads, uint32_t ppl, bool repair,
                            bool single, bool hold);
const void *spec_wave_kernel_for(uint32_t fam, bool repair, uint32_t windows);
const void *single_kernel_for(uint32_t fam);
const void *spec_words_kernel_for(uint32_t fam, bool repair);
const void *triple_kernel_for(uint32_t fam, bool seq);
const void *counted_triple_kernel_for(uint32_t fam, bool produce);
const void *chunk_kernel_for(uint32_t fam, bool repair, uint32_t cpw);
const void *chunk_prep_kernel_ptr();
const void *counted_kernel_for(uint32_t fam, bool produce);
const void *counted_scan_kernel_ptr(bool top);
hipError_t launch_toggle_flip(uint32_t *flip, hipStream_t stream);
const void *toggle_flip_kernel_ptr();
hipError_t launch_fill(const void *kernel, uint32_t grid, uint32_t threads,
                       const LaunchArgs &args, hipStream_t stream);
hipError_t launch_expand_tiles(const Segment *segs, uint32_t nseg, uint32_t *tile_seg,
                               hipStream_t stream);
hipError_t launch_set_counter(uint64_t *slot, uint64_t value, hipStream_t stream);
hipError_t launch_ranmar_set(const RanmarInit &r, hipStream_t stream);
hipError_t launch_ranmar_set_many(const RanmarInit *inits, uint32_t count, hipStream_t stream);
const void *ranmar_kernel_for(uint32_t fam, uint32_t mode);
hipError_t launch_zero_words(uint64_t *p, size_t n, hipStream_t stream);
hipError_t noalloc_setup(int dev);
Control *noalloc_control(int dev);
uint64_t *noalloc_status(int dev);
size_t noalloc_status_words();
}  // namespace prngd

using namespace prngd;

namespace {

// ----------------------------------------------------------------- errors
thread_local std::string g_last_error;

// Polls of a look-back wait before it reports a stall, for launches
// planned from now on (0: the default); set by prngd_probe_set_spin_limit.
std::atomic<uint32_t> g_spin_limit{0};

prngd_status_t fail(prngd_status_t st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

prngd_status_t hip_fail(hipError_t e, const char *what)
{
    return fail(PRNGD_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess)                           \
            return hip_fail(e_, #expr);                 \
    } while (0)

std::recursive_mutex g_mutex;

// ------------------------------------------------------------ constants
constexpr uint64_t kM1 = 4294967087ull;
constexpr uint64_t kM2 = 4294944443ull;

struct Config {
    uint32_t fam;
    uint32_t w;
    uint64_t a0, a, b0, b;
    uint64_t D;
    double S;
    uint32_t map;     // prngd_map_t
    uint32_t consume; // prngd_consume_t
    uint64_t D4;      // Eq. (4) denominator in integer units: (a - a0) 2^w - (b - b0)
    double S4;        // RN(1 / D4)
    uint32_t arity;   // words per output: 2, or 3 (the two-word method applied twice)
    double S3;        // three words: RN((1 - 2^-3w) / D3)
};

// The map constants a launch passes to the kernels.
struct MapConsts {
    double S, nadd, osign, ooff;
};

// RN((1 - 2^-2w) / D): long division of (2^2w - 1) by D to 64 significant
// bits plus a sticky bit, rounded half-to-even to 53 bits, scaled by 2^-2w.
// (2^2w - 1) > D for every valid configuration, so the quotient is >= 1.
double folded_constant(uint32_t w, uint64_t D)
{
    const uint64_t num = w == 32 ? ~uint64_t(0) : (uint64_t(1) << (2 * w)) - 1;
    uint64_t q = num / D;
    uint64_t r = num % D;
    int bits = 64 - __builtin_clzll(q);
    int frac = 0;
    while (bits + frac < 64) {
        const unsigned __int128 r2 = static_cast<unsigned __int128>(r) << 1;
        const bool bit = r2 >= D;
        r = static_cast<uint64_t>(bit ? r2 - D : r2);
        q = (q << 1) | uint64_t(bit);
        ++frac;
    }
    uint64_t keep = q >> 11;
    const uint64_t dropped = q & 0x7FFu;
    const bool sticky = r != 0;
    if (dropped > 0x400u || (dropped == 0x400u && (sticky || (keep & 1u))))
        ++keep;
    return std::ldexp(static_cast<double>(keep), 11 - frac - int(2 * w));
}

// RN(1 / D) for D >= 2: 2^(62 + L) / D with L the bit length of D has 63
// or 64 significant bits; rounded half-to-even to 53 with the remainder as
// sticky bit.
double folded_recip(uint64_t D)
{
    const int L = 64 - __builtin_clzll(D);
    const int sh = 62 + L;
    const unsigned __int128 num = static_cast<unsigned __int128>(1) << sh;
    const uint64_t q = static_cast<uint64_t>(num / D);
    const bool sticky = (num % D) != 0;
    const int bits = 64 - __builtin_clzll(q);
    const int drop = bits - 53;
    uint64_t keep = q >> drop;
    const uint64_t dropped = q & ((uint64_t(1) << drop) - 1);
    const uint64_t half = uint64_t(1) << (drop - 1);
    if (dropped > half || (dropped == half && (sticky || (keep & 1u))))
        ++keep;
    return std::ldexp(static_cast<double>(keep), drop - sh);
}

// RN((1 - 2^-3w) / D3) for 0 < D3 < 2^3w <= 2^96: (2^3w - 1) / D3 by long
// division in 31-bit digits (each step divides a remainder below 2^127),
// until 64 significant quotient bits are known; then rounded half-to-even to
// 53 bits with the last remainder as sticky bit.
double folded_constant3(uint32_t w, unsigned __int128 D3)
{
    const unsigned __int128 num = (static_cast<unsigned __int128>(1) << (3 * w)) - 1;
    unsigned __int128 q = num / D3;   // integer part: 1 .. 2^3w
    unsigned __int128 r = num % D3;
    int frac = 0;
    auto bits_of = [](unsigned __int128 x) {
        int b = 0;
        while (x) {
            ++b;
            x >>= 1;
        }
        return b;
    };
    while (bits_of(q) < 64) {
        const unsigned __int128 r2 = r << 31;
        q = (q << 31) | (r2 / D3);
        r = r2 % D3;
        frac += 31;
    }
    const int drop = bits_of(q) - 53;
    uint64_t keep = static_cast<uint64_t>(q >> drop);
    const unsigned __int128 dropped = q & ((static_cast<unsigned __int128>(1) << drop) - 1);
    const unsigned __int128 half = static_cast<unsigned __int128>(1) << (drop - 1);
    if (dropped > half || (dropped == half && (r != 0 || (keep & 1u))))
        ++keep;
    return std::ldexp(static_cast<double>(keep), drop - frac - int(3 * w));
}

// D3 = (a - a0 - 2) 2^2w + (a - a0 - 2) 2^w + (a - a0): the Eq. (5)
// denominator of three words per output, in integer units.
unsigned __int128 triple_denominator(const Config &c)
{
    const unsigned __int128 span = c.a - c.a0;
    return ((span - 2) << (2 * c.w)) + ((span - 2) << c.w) + span;
}

MapConsts map_consts(const Config &c)
{
    if (c.arity == 3)
        return {c.S3, 0.0, 1.0, 0.0};
    if (c.map == PRNGD_MAP_EQ4)
        return {c.S4, double((uint64_t(1) << c.w) - (c.b - c.b0)), 1.0, 0.0};
    if (c.map == PRNGD_MAP_ONE_MINUS)
        return {c.S, 0.0, -1.0, 1.0};
    return {c.S, 0.0, 1.0, 0.0};
}

// The kernel family that serves a generator at resolution 2^-w.
uint32_t kernel_family(prngd_generator_t gen, uint32_t w)
{
    switch (gen) {
    case PRNGD_MRG32K3A: return FAM_MRG;
    case PRNGD_PHILOX_X1_MRG32K3A_X2: return FAM_MIXED;
    case PRNGD_ENUMERATE: return FAM_ENUM;
    case PRNGD_RANMAR: return FAM_RANMAR;
    default: return w == 32 ? FAM_PHILOX32 : FAM_PHILOX;
    }
}

prngd_status_t make_config(prngd_generator_t gen, double k, uint64_t min, uint64_t max,
                           Config *c)
{
    if (gen < PRNGD_PHILOX4X32_10 || gen > PRNGD_RANMAR)
        return fail(PRNGD_ERR_UNSUPPORTED, "unknown generator %d", int(gen));
    if (!(k > 0) || !std::isfinite(k))
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "k must be 2^-w");
    int e = 0;
    const double m = std::frexp(k, &e);
    if (m != 0.5)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "k = %a is not a power of two", k);
    const int w = 1 - e;
    c->w = uint32_t(w);
    const int wmax = gen == PRNGD_ENUMERATE ? 16 : gen == PRNGD_RANMAR ? 24 : 32;
    const int wmin = (gen == PRNGD_MRG32K3A || gen == PRNGD_PHILOX_X1_MRG32K3A_X2) ? 32
                     : gen == PRNGD_RANMAR                                         ? 24
                                                                                   : 2;
    if (w < wmin || w > wmax)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "k = 2^-%d out of range for this generator", w);
    const uint64_t top = (uint64_t(1) << w) - 1;
    switch (gen) {
    case PRNGD_PHILOX4X32_10:
    case PRNGD_ENUMERATE:
    case PRNGD_RANMAR:
        c->a0 = 0; c->a = top; c->b0 = 0; c->b = top;
        break;
    case PRNGD_MRG32K3A:
        c->a0 = 1; c->a = kM1; c->b0 = 1; c->b = kM1;
        break;
    default:
        c->a0 = 0; c->a = top; c->b0 = 1; c->b = kM1;
        break;
    }
    if (min != c->a0 || max != c->a)
        return fail(PRNGD_ERR_INVALID_ARGUMENT,
                    "[min, max] = [%llu, %llu] must be the generator's range [%llu, %llu]",
                    (unsigned long long)min, (unsigned long long)max,
                    (unsigned long long)c->a0, (unsigned long long)c->a);
    c->D = (c->a - c->a0 - 2) * (uint64_t(1) << w) + (c->b - c->b0);
    c->S = folded_constant(c->w, c->D);
    c->D4 = (c->a - c->a0) * (uint64_t(1) << w) - (c->b - c->b0);
    c->S4 = folded_recip(c->D4);
    c->map = PRNGD_MAP_EQ5;
    c->consume = PRNGD_CONSUME_PAIR;
    c->fam = kernel_family(gen, c->w);
    c->arity = 2;
    c->S3 = 0.0;
    return PRNGD_OK;
}

// ---------------------------------------------------- MRG32k3a matrices
struct Mat {
    uint64_t e[9];
};

Mat mat_identity()
{
    return Mat{{1, 0, 0, 0, 1, 0, 0, 0, 1}};
}

Mat mat_mul(const Mat &x, const Mat &y, uint64_t m)
{
    Mat z;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            unsigned __int128 s = 0;
            for (int l = 0; l < 3; ++l)
                s += static_cast<unsigned __int128>(x.e[3 * i + l]) * y.e[3 * l + j];
            z.e[3 * i + j] = static_cast<uint64_t>(s % m);
        }
    return z;
}

// The companion matrices of the two recurrences of L'Ecuyer's MRG32k3a
// acting on (x[n-3], x[n-2], x[n-1]).
Mat mrg_step_matrix(int comp)
{
    if (comp == 0)
        return Mat{{0, 1, 0, 0, 0, 1, kM1 - 810728, 1403580, 0}};
    return Mat{{0, 1, 0, 0, 0, 1, kM2 - 1370589, 0, 527612}};
}

Mat mat_pow(Mat base, uint64_t e, uint64_t m)
{
    Mat r = mat_identity();
    while (e) {
        if (e & 1)
            r = mat_mul(r, base, m);
        base = mat_mul(base, base, m);
        e >>= 1;
    }
    return r;
}

Mat mat_pow2k(Mat base, int k, uint64_t m)   // base^(2^k)
{
    for (int i = 0; i < k; ++i)
        base = mat_mul(base, base, m);
    return base;
}

void mat_apply(const Mat &M, uint32_t *v, uint64_t m)
{
    uint64_t r[3];
    for (int i = 0; i < 3; ++i) {
        unsigned __int128 s = 0;
        for (int l = 0; l < 3; ++l)
            s += static_cast<unsigned __int128>(M.e[3 * i + l]) * v[l];
        r[i] = static_cast<uint64_t>(s % m);
    }
    for (int i = 0; i < 3; ++i)
        v[i] = uint32_t(r[i]);
}

// Powers A^(2^127 * 2^i) (i < 64) and A^(2^76 * 2^i) (i < 32) per component.
struct StreamJumps {
    Mat seq[2][64];
    Mat sub[2][32];
    StreamJumps()
    {
        for (int c = 0; c < 2; ++c) {
            const uint64_t m = c == 0 ? kM1 : kM2;
            Mat p = mat_pow2k(mrg_step_matrix(c), 76, m);
            for (int i = 0; i < 32; ++i) {
                sub[c][i] = p;
                p = mat_mul(p, p, m);
            }
            p = mat_pow2k(mrg_step_matrix(c), 127, m);
            for (int i = 0; i < 64; ++i) {
                seq[c][i] = p;
                p = mat_mul(p, p, m);
            }
        }
    }
};

const StreamJumps &stream_jumps()
{
    static const StreamJumps j;
    return j;
}

// State at position 0 of substream (seed, stream): 12345 six times advanced
// by seed * 2^127 + stream * 2^76 steps (L'Ecuyer et al. 2002 streams and
// substreams).
void mrg_stream_base(uint64_t seed, uint32_t stream, uint32_t out[6])
{
    const StreamJumps &J = stream_jumps();
    for (int i = 0; i < 6; ++i)
        out[i] = 12345u;
    for (int c = 0; c < 2; ++c) {
        const uint64_t m = c == 0 ? kM1 : kM2;
        for (int i = 0; i < 64; ++i)
            if ((seed >> i) & 1u)
                mat_apply(J.seq[c][i], out + 3 * c, m);
        for (int i = 0; i < 32; ++i)
            if ((stream >> i) & 1u)
                mat_apply(J.sub[c][i], out + 3 * c, m);
    }
}

void put_entry(uint32_t *dst, const Mat &m1, const Mat &m2)
{
    for (int i = 0; i < 9; ++i) {
        dst[i] = uint32_t(m1.e[i]);
        dst[9 + i] = uint32_t(m2.e[i]);
    }
}

// Jump tables of the MRG kernels for `r` MRG outputs per pair and
// pairs-per-lane `ppl`: thread[tid] = A^(r ppl tid), window[d][v] =
// A^(r T v 256^d) with T = 256 ppl.
void build_mrg_tables(uint32_t r, uint32_t ppl, std::vector<uint32_t> &thread,
                      std::vector<uint32_t> &window)
{
    thread.assign(size_t(kMrgBlockThreads) * kMrgMatWords, 0);
    window.assign(size_t(kMrgDigits) * 256 * kMrgMatWords, 0);
    const uint64_t T = uint64_t(kMrgBlockThreads) * ppl;
    Mat step[2], cur[2];
    for (int c = 0; c < 2; ++c) {
        const uint64_t m = c == 0 ? kM1 : kM2;
        step[c] = mat_pow(mrg_step_matrix(c), uint64_t(r) * ppl, m);
        cur[c] = mat_identity();
    }
    for (int t = 0; t < kMrgBlockThreads; ++t) {
        put_entry(&thread[size_t(t) * kMrgMatWords], cur[0], cur[1]);
        cur[0] = mat_mul(cur[0], step[0], kM1);
        cur[1] = mat_mul(cur[1], step[1], kM2);
    }
    Mat digit_base[2];
    for (int c = 0; c < 2; ++c)
        digit_base[c] = mat_pow(mrg_step_matrix(c), uint64_t(r) * T, c == 0 ? kM1 : kM2);
    for (int d = 0; d < kMrgDigits; ++d) {
        Mat acc[2] = {mat_identity(), mat_identity()};
        for (int v = 0; v < 256; ++v) {
            put_entry(&window[(size_t(d) * 256 + v) * kMrgMatWords], acc[0], acc[1]);
            acc[0] = mat_mul(acc[0], digit_base[0], kM1);
            acc[1] = mat_mul(acc[1], digit_base[1], kM2);
        }
        // digit_base <- digit_base^256
        for (int c = 0; c < 2; ++c)
            digit_base[c] = mat_pow2k(digit_base[c], 8, c == 0 ? kM1 : kM2);
    }
}

// ---------------------------------------------------------- device info
struct DeviceInfo {
    int cus = 0;
    uint32_t *error_host = nullptr;      // mapped pinned word
    uint32_t *error_dev = nullptr;
    uint32_t *zero_word = nullptr;       // device word that stays 0 (replay parity of
                                         // launches outside plans)
    std::vector<uint64_t *> slot_chunks;
    std::vector<uint64_t *> clean_slots;   // zero since their chunk was cleared
    std::vector<uint64_t *> free_slots;    // returned by destroyed handles
    std::map<std::pair<uint32_t, uint32_t>, std::pair<uint32_t *, uint32_t *>> mrg_tables;
    std::map<const void *, int> occupancy;
    // prngd_fill_noalloc: launches made on the fixed scratch, and the event
    // recorded after each (both set up here, never by the entry point)
    uint64_t noalloc_launches = 0;
    hipEvent_t noalloc_event = nullptr;
    // RANMAR: handle states from slabs, and the jump table of the fills'
    // segments (rows of kRanmarRow words)
    std::vector<void *> rm_slabs;
    std::vector<RanmarState *> rm_free;
    uint32_t *rm_jump[2] = {nullptr, nullptr};    // fine and coarse segments
    uint32_t rm_jump_rows[2] = {0, 0};
    std::vector<uint32_t> rm_jump_host[2];
};

std::map<int, DeviceInfo> g_devices;

prngd_status_t device_info(int dev, DeviceInfo **out)
{
    auto it = g_devices.find(dev);
    if (it != g_devices.end()) {
        *out = &it->second;
        return PRNGD_OK;
    }
    DeviceInfo d;
    HIP_TRY(hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev));
    void *p = nullptr;
    HIP_TRY(hipHostMalloc(&p, 64, hipHostMallocMapped | hipHostMallocCoherent));
    d.error_host = static_cast<uint32_t *>(p);
    *d.error_host = 0;
    void *dp = nullptr;
    HIP_TRY(hipHostGetDevicePointer(&dp, p, 0));
    d.error_dev = static_cast<uint32_t *>(dp);
    HIP_TRY(hipMalloc(&dp, 256));
    HIP_TRY(hipMemset(dp, 0, 256));
    d.zero_word = static_cast<uint32_t *>(dp);
    // the fixed scratch of prngd_fill_noalloc, with this device current
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != dev)
        HIP_TRY(hipSetDevice(dev));
    const hipError_t se = noalloc_setup(dev);
    if (se == hipSuccess && cur != dev)
        HIP_TRY(hipSetDevice(cur));
    HIP_TRY(se);
    HIP_TRY(hipEventCreateWithFlags(&d.noalloc_event, hipEventDisableTiming));
    *out = &g_devices.emplace(dev, std::move(d)).first->second;
    return PRNGD_OK;
}

prngd_status_t check_device_errors(DeviceInfo *d)
{
    const uint32_t e = __atomic_load_n(d->error_host, __ATOMIC_ACQUIRE);
    if (e) {
        __atomic_store_n(d->error_host, 0u, __ATOMIC_RELEASE);
        return fail(PRNGD_ERR_DEVICE, "a previous fill reported device error 0x%x", e);
    }
    return PRNGD_OK;
}

// Position slots (two 64-bit counters) come from 4096-slot chunks; a slot
// handed out again after its handle was destroyed is zeroed first.
prngd_status_t alloc_slot(DeviceInfo *d, uint64_t **slot)
{
    if (d->clean_slots.empty() && d->free_slots.empty()) {
        constexpr size_t kChunk = 4096;
        void *p = nullptr;
        HIP_TRY(hipMalloc(&p, kChunk * 2 * sizeof(uint64_t)));
        HIP_TRY(hipMemset(p, 0, kChunk * 2 * sizeof(uint64_t)));
        HIP_TRY(hipDeviceSynchronize());
        uint64_t *base = static_cast<uint64_t *>(p);
        d->slot_chunks.push_back(base);
        for (size_t i = kChunk; i-- > 0;)
            d->clean_slots.push_back(base + 2 * i);
    }
    if (!d->clean_slots.empty()) {
        *slot = d->clean_slots.back();
        d->clean_slots.pop_back();
        return PRNGD_OK;
    }
    uint64_t *s = d->free_slots.back();
    const uint64_t zero[2] = {0, 0};
    HIP_TRY(hipMemcpy(s, zero, sizeof zero, hipMemcpyHostToDevice));
    d->free_slots.pop_back();
    *slot = s;
    return PRNGD_OK;
}

// RANMAR handle states come from slabs of 1024 (1 KB each).
prngd_status_t alloc_ranmar(DeviceInfo *d, RanmarState **out)
{
    if (d->rm_free.empty()) {
        constexpr size_t kSlab = 1024;
        void *p = nullptr;
        HIP_TRY(hipMalloc(&p, kSlab * sizeof(RanmarState)));
        d->rm_slabs.push_back(p);
        RanmarState *base = static_cast<RanmarState *>(p);
        for (size_t i = kSlab; i-- > 0;)
            d->rm_free.push_back(base + i);
    }
    *out = d->rm_free.back();
    d->rm_free.pop_back();
    return PRNGD_OK;
}

// The states of new RANMAR handles at word 0 of their streams, set at once
// (a staging copy and one kernel, then a wait: handle creation only).
prngd_status_t ranmar_init_states(const std::vector<std::pair<RanmarState *, const void *>> &hs,
                                  uint64_t seed, uint32_t first_stream)
{
    std::vector<RanmarInit> inits(hs.size());
    for (size_t i = 0; i < hs.size(); ++i) {
        inits[i].dst = hs[i].first;
        inits[i].slot = nullptr;
        inits[i].counter = 0;
        ranmar_window_at(seed, uint32_t(first_stream + i), 0, 0, inits[i].words);
    }
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, inits.size() * sizeof(RanmarInit)));
    hipError_t e = hipMemcpy(p, inits.data(), inits.size() * sizeof(RanmarInit),
                             hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = launch_ranmar_set_many(static_cast<RanmarInit *>(p), uint32_t(inits.size()), nullptr);
    if (e == hipSuccess)
        e = hipDeviceSynchronize();
    (void)hipFree(p);
    HIP_TRY(e);
    return PRNGD_OK;
}

prngd_status_t mrg_tables_for(DeviceInfo *d, uint32_t r, uint32_t ppl, const uint32_t **thread,
                              const uint32_t **window, bool may_alloc = true)
{
    auto key = std::make_pair(r, ppl);
    auto it = d->mrg_tables.find(key);
    if (it == d->mrg_tables.end()) {
        if (!may_alloc)
            return fail(PRNGD_ERR_UNSUPPORTED, "no MRG32k3a jump tables for %u pairs per lane "
                                               "yet: they are built by prngd_fill", ppl);
        std::vector<uint32_t> th, wi;
        build_mrg_tables(r, ppl, th, wi);
        void *pt = nullptr, *pw = nullptr;
        HIP_TRY(hipMalloc(&pt, th.size() * 4));
        HIP_TRY(hipMalloc(&pw, wi.size() * 4));
        HIP_TRY(hipMemcpy(pt, th.data(), th.size() * 4, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(pw, wi.data(), wi.size() * 4, hipMemcpyHostToDevice));
        it = d->mrg_tables.emplace(key, std::make_pair(static_cast<uint32_t *>(pt),
                                                       static_cast<uint32_t *>(pw))).first;
    }
    *thread = it->second.first;
    *window = it->second.second;
    return PRNGD_OK;
}

// ---------------------------------------------------------------- tuning
std::map<std::pair<uint32_t, uint32_t>, prngd_tuning_t> g_tuning;

bool philox_family(uint32_t fam)
{
    return fam == FAM_PHILOX || fam == FAM_ENUM || fam == FAM_PHILOX32;
}

// The launch shape for (family, w): the tuning set for it, library
// defaults in its zero fields (default_ppl pairs per lane).
prngd_tuning_t tuning_for(uint32_t fam, uint32_t w, uint32_t default_ppl = 16)
{
    prngd_tuning_t t{};
    auto it = g_tuning.find(std::make_pair(fam, w));
    if (it != g_tuning.end())
        t = it->second;
    if (t.block_threads == 0)
        t.block_threads = philox_family(fam) ? 256 : kMrgBlockThreads;
    if (t.pairs_per_lane == 0)
        t.pairs_per_lane = default_ppl;
    return t;
}

// Whether no pairs-per-lane value has been set for (family, w).
bool ppl_is_default(uint32_t fam, uint32_t w)
{
    auto it = g_tuning.find(std::make_pair(fam, w));
    return it == g_tuning.end() || it->second.pairs_per_lane == 0;
}

// Default pairs per lane of a single Philox fill on a tile-speculative
// path: 2048-pair tiles measured fastest on MI355X there (batches keep 16);
// on the wave-granular path, chunks of one 128-pair window.
constexpr uint32_t kSingleSpecPpl = 8;
constexpr uint32_t kSingleWavePpl = 2;

// Segments of a batch with at most this many tiles are produced whole by
// one workgroup (segment-sequential kernel); longer ones are spread over
// workgroups and joined by the look-back.  Default: a segment may take up
// to half a workgroup's fair share of the batch.
uint64_t seq_limit(const prngd_tuning_t &t, uint64_t total_tiles, uint64_t workgroups)
{
    if (t.seq_max_tiles)
        return t.seq_max_tiles;
    return std::max<uint64_t>(4, total_tiles / std::max<uint64_t>(1, 2 * workgroups));
}

// ------------------------------------------------------------ workspaces
// Launch control and tile status words for launches that follow each
// other in stream order (one per stream, one per plan).
struct Workspace {
    int device = 0;
    Control *ctl = nullptr;               // look-back kernel
    Control *seq_ctl = nullptr;           // segment-sequential kernel
    uint64_t *status = nullptr;
    size_t status_cap = 0;
    // speculative fill: list control, rejection list, per-tile hints
    SpecControl *spec = nullptr;
    uint64_t *rejlist = nullptr;
    uint32_t *hint = nullptr;
    size_t spec_cap = 0;
    uint64_t *hint64 = nullptr;           // wave-granular form: per chunk
    size_t hint64_cap = 0;
    uint64_t spec_epoch = 0;
    // chunk-speculative batch form: per segment record, first dirty chunk
    // (zero between launches) and the list of dirty segments
    ChunkSeg *chunk_segs = nullptr;
    uint32_t *first_dirty = nullptr;
    uint32_t *dirty_list = nullptr;
    size_t chunk_cap = 0;
    // counted single fill: per-chunk counts and offsets, per-block offsets
    uint32_t *counts = nullptr;
    uint32_t *count_offs = nullptr;
    uint64_t *block_offs = nullptr;
    size_t counts_cap = 0;
    // buffers replaced by larger ones: kept until the workspace is released,
    // so that growing never waits for work in flight (freeing would)
    std::vector<void *> retired_dev;
    std::vector<void *> retired_host;
    uint64_t launches = 0;
    hipEvent_t last = nullptr;            // recorded after every launch
    // batch descriptors and the tile -> segment map
    Segment *dsegs = nullptr;
    size_t dsegs_cap = 0;
    uint32_t *tile_seg = nullptr;
    size_t tile_seg_cap = 0;
    Segment *hsegs[2] = {nullptr, nullptr};
    size_t hsegs_cap[2] = {0, 0};
    hipEvent_t hsegs_done[2] = {nullptr, nullptr};
    int hcur = 0;
};

prngd_status_t ws_init(Workspace *ws, int dev)
{
    ws->device = dev;
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, 2 * sizeof(Control)));
    ws->ctl = static_cast<Control *>(p);
    ws->seq_ctl = ws->ctl + 1;
    Control init[2];
    std::memset(init, 0, sizeof init);
    init[0].epoch = 1;
    init[1].epoch = 1;
    HIP_TRY(hipMemcpy(ws->ctl, init, sizeof init, hipMemcpyHostToDevice));
    HIP_TRY(hipMalloc(&p, sizeof(SpecControl)));
    ws->spec = static_cast<SpecControl *>(p);
    HIP_TRY(hipMemset(ws->spec, 0, sizeof(SpecControl)));
    HIP_TRY(hipEventCreateWithFlags(&ws->last, hipEventDisableTiming));
    for (int i = 0; i < 2; ++i)
        HIP_TRY(hipEventCreateWithFlags(&ws->hsegs_done[i], hipEventDisableTiming));
    return PRNGD_OK;
}

void ws_release(Workspace *ws)
{
    for (void *p : ws->retired_dev)
        (void)hipFree(p);
    for (void *p : ws->retired_host)
        (void)hipHostFree(p);
    (void)hipFree(ws->status);
    (void)hipFree(ws->ctl);
    (void)hipFree(ws->spec);
    (void)hipFree(ws->rejlist);
    (void)hipFree(ws->hint);
    (void)hipFree(ws->hint64);
    (void)hipFree(ws->chunk_segs);
    (void)hipFree(ws->first_dirty);
    (void)hipFree(ws->dirty_list);
    (void)hipFree(ws->counts);
    (void)hipFree(ws->count_offs);
    (void)hipFree(ws->block_offs);
    (void)hipFree(ws->dsegs);
    (void)hipFree(ws->tile_seg);
    for (int i = 0; i < 2; ++i) {
        if (ws->hsegs[i])
            (void)hipHostFree(ws->hsegs[i]);
        (void)hipEventDestroy(ws->hsegs_done[i]);
    }
    (void)hipEventDestroy(ws->last);
}

// Make room for `tiles` status words and clear them when the 24-bit epoch
// wraps, so that no stale word can carry the epoch of a later launch.
prngd_status_t ws_prepare(Workspace *ws, size_t tiles, hipStream_t stream)
{
    if (tiles > ws->status_cap) {
        const size_t cap = std::max<size_t>({tiles, size_t(1) << 16, 2 * ws->status_cap});
        if (ws->status) {
            ws->retired_dev.push_back(ws->status);
            ws->status = nullptr;
        }
        void *p = nullptr;
        HIP_TRY(hipMalloc(&p, cap * sizeof(uint64_t)));
        ws->status = static_cast<uint64_t *>(p);
        ws->status_cap = cap;
        HIP_TRY(launch_zero_words(ws->status, cap, stream));
    }
    if (ws->launches > 0 && ws->launches % kEpochMask == 0)
        HIP_TRY(launch_zero_words(ws->status, ws->status_cap, stream));
    return PRNGD_OK;
}

// Make room for the speculative fill's rejection list and hints of `tiles`
// tiles.  A new list starts empty (all slots zero); afterwards every
// repair launch leaves it empty again.
prngd_status_t ws_prepare_spec(Workspace *ws, size_t tiles, hipStream_t stream)
{
    if (tiles <= ws->spec_cap)
        return PRNGD_OK;
    const size_t cap = std::max<size_t>({tiles, size_t(1) << 20, 2 * ws->spec_cap});
    if (ws->rejlist) {
        ws->retired_dev.push_back(ws->rejlist);
        ws->retired_dev.push_back(ws->hint);
        ws->rejlist = nullptr;
        ws->hint = nullptr;
    }
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, cap * sizeof(uint64_t)));
    ws->rejlist = static_cast<uint64_t *>(p);
    HIP_TRY(hipMalloc(&p, cap * sizeof(uint32_t)));
    ws->hint = static_cast<uint32_t *>(p);
    ws->spec_cap = cap;
    HIP_TRY(launch_zero_words(ws->rejlist, cap, stream));
    return PRNGD_OK;
}

// Room for the wave-granular form's per-chunk hints (never cleared: a
// record counts only while it carries the current launch epoch).
prngd_status_t ws_prepare_hint64(Workspace *ws, size_t chunks, hipStream_t stream)
{
    if (chunks <= ws->hint64_cap)
        return PRNGD_OK;
    const size_t cap = std::max<size_t>({chunks, size_t(1) << 20, 2 * ws->hint64_cap});
    if (ws->hint64) {
        ws->retired_dev.push_back(ws->hint64);
        ws->hint64 = nullptr;
    }
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, cap * sizeof(uint64_t)));
    ws->hint64 = static_cast<uint64_t *>(p);
    ws->hint64_cap = cap;
    HIP_TRY(launch_zero_words(ws->hint64, cap, stream));
    return PRNGD_OK;
}

// Room for the chunk-speculative batch form's per-segment buffers of
// `nseg` segments.  A new first-dirty array starts zero; afterwards every
// repair launch leaves it zero again.
prngd_status_t ws_prepare_chunk(Workspace *ws, size_t nseg, hipStream_t stream)
{
    if (nseg <= ws->chunk_cap)
        return PRNGD_OK;
    // even, so that the first-dirty array is whole 8-byte words
    const size_t cap = (std::max<size_t>({nseg, size_t(1024), 2 * ws->chunk_cap}) + 1) & ~size_t(1);
    if (ws->chunk_segs) {
        ws->retired_dev.push_back(ws->chunk_segs);
        ws->retired_dev.push_back(ws->first_dirty);
        ws->retired_dev.push_back(ws->dirty_list);
        ws->chunk_segs = nullptr;
        ws->first_dirty = nullptr;
        ws->dirty_list = nullptr;
    }
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, cap * sizeof(ChunkSeg)));
    ws->chunk_segs = static_cast<ChunkSeg *>(p);
    HIP_TRY(hipMalloc(&p, cap * sizeof(uint32_t)));
    ws->first_dirty = static_cast<uint32_t *>(p);
    HIP_TRY(hipMalloc(&p, cap * sizeof(uint32_t)));
    ws->dirty_list = static_cast<uint32_t *>(p);
    ws->chunk_cap = cap;
    HIP_TRY(launch_zero_words(reinterpret_cast<uint64_t *>(ws->first_dirty), cap / 2, stream));
    return PRNGD_OK;
}

// Room for the counted fill's per-chunk counts and offsets of `chunks`
// chunks (and its fixed per-block offsets).
prngd_status_t ws_prepare_counted(Workspace *ws, size_t chunks)
{
    if (!ws->block_offs) {
        void *p = nullptr;
        HIP_TRY(hipMalloc(&p, kScanBlocksMax * sizeof(uint64_t)));
        ws->block_offs = static_cast<uint64_t *>(p);
    }
    if (chunks <= ws->counts_cap)
        return PRNGD_OK;
    const size_t cap = std::max<size_t>({chunks, size_t(1) << 16, 2 * ws->counts_cap});
    if (ws->counts) {
        ws->retired_dev.push_back(ws->counts);
        ws->retired_dev.push_back(ws->count_offs);
        ws->counts = nullptr;
        ws->count_offs = nullptr;
    }
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, cap * sizeof(uint32_t)));
    ws->counts = static_cast<uint32_t *>(p);
    HIP_TRY(hipMalloc(&p, cap * sizeof(uint32_t)));
    ws->count_offs = static_cast<uint32_t *>(p);
    ws->counts_cap = cap;
    return PRNGD_OK;
}

// Grow a device buffer that only work on `stream` (or the workspace's
// earlier launches) uses.
template <class T>
prngd_status_t ws_grow(Workspace *ws, T **buf, size_t *cap, size_t need, hipStream_t stream)
{
    if (*cap >= need)
        return PRNGD_OK;
    (void)stream;
    if (*buf) {
        ws->retired_dev.push_back(*buf);
        *buf = nullptr;
    }
    const size_t c = std::max<size_t>({need, size_t(1024), 2 * *cap});
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, c * sizeof(T)));
    *buf = static_cast<T *>(p);
    *cap = c;
    return PRNGD_OK;
}

std::map<std::pair<int, hipStream_t>, std::unique_ptr<Workspace>> g_stream_ws;

prngd_status_t stream_workspace(int dev, hipStream_t stream, Workspace **out)
{
    auto key = std::make_pair(dev, stream);
    auto it = g_stream_ws.find(key);
    if (it == g_stream_ws.end()) {
        std::unique_ptr<Workspace> ws(new Workspace);
        prngd_status_t st = ws_init(ws.get(), dev);
        if (st != PRNGD_OK)
            return st;
        it = g_stream_ws.emplace(key, std::move(ws)).first;
    }
    *out = it->second.get();
    return PRNGD_OK;
}

}  // namespace

// ----------------------------------------------------------------- handle
struct prngd_handle_s {
    int device = 0;
    prngd_generator_t gen = PRNGD_PHILOX4X32_10;
    Config cfg{};
    uint64_t seed = 0;
    uint32_t stream_id = 0;
    uint32_t mrg[6] = {0, 0, 0, 0, 0, 0};
    uint64_t *slot = nullptr;          // device: counter[2]
    RanmarState *rm = nullptr;         // device: RANMAR state slots (RANMAR handles)
    uint32_t parity = 0;               // counter[parity] is current
    hipEvent_t last_event = nullptr;   // borrowed: last work on this handle
    hipStream_t last_stream = nullptr;
    prngd_plan_s *plan = nullptr;      // live plan the handle is bound to
    size_t plan_index = 0;             // position in that plan
};

struct prngd_plan_s {
    int device = 0;
    std::vector<prngd_handle_t> handles;
    std::vector<uint32_t> base_parity;
    Workspace ws;
    Segment *dsegs = nullptr;          // look-back segments, then sequential ones
    uint32_t *tile_seg = nullptr;
    uint32_t *flip = nullptr;          // device word: parity of the next replay
    LaunchArgs lb_args{};
    LaunchArgs seq_args{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t launches = 0;
    bool spec = false;                 // speculative fill (no status words)
};

namespace {

// Order work on `stream` after the handle's previous work elsewhere.
prngd_status_t order_after(prngd_handle_t h, hipStream_t stream)
{
    if (h->last_event && h->last_stream != stream)
        HIP_TRY(hipStreamWaitEvent(stream, h->last_event, 0));
    return PRNGD_OK;
}

uint64_t planned_pairs(const Config &c, uint64_t n, uint32_t slack_mode)
{
    if (slack_mode == 1)
        return n;
    // expected rejections before n acceptances (x1 uniform on [a0, a]; with
    // three words per output x1 and x2 are tested)
    const double r1 = 2.0 / double(c.a - c.a0 + 1);
    const double rho = c.arity == 3 ? 1.0 - (1.0 - r1) * (1.0 - r1) : r1;
    const double mean = double(n) * rho / (1.0 - rho);
    const double extra = std::floor(mean + 4.0 * std::sqrt(mean) + 0.5);
    return n + static_cast<uint64_t>(extra);
}

int occupancy_of(DeviceInfo *d, const void *kernel, uint32_t threads)
{
    auto it = d->occupancy.find(kernel);
    if (it != d->occupancy.end())
        return it->second;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, int(threads), 0) !=
            hipSuccess || nb <= 0)
        nb = 1;
    d->occupancy[kernel] = nb;
    return nb;
}

// Kernels, tile size and generator constants of one launch.
struct LaunchPlan {
    const void *kernel;       // look-back kernel
    const void *seq_kernel;   // segment-sequential kernel
    const void *spec_kernels[2][2];  // [holding form][single segment]
    const void *spec_kernel;  // the chosen speculative fill (batches, single
    const void *spec_single_kernel;  // fills) and its repair
    const void *repair_kernel;
    const void *wave_kernel;  // wave-granular single-segment form, if any
    const void *wave_repair_kernel;
    const void *words_kernel;         // one-word consumption across workgroups
    const void *words_repair_kernel;
    const void *chunk_kernel;         // chunk-speculative batch form, if any
    const void *chunk_repair_kernel;
    bool wave;                // single fills take the wave-granular form
    const void *counted_kernels[2];   // counted single fill: count, produce
    bool counted_triples;     // ... of three words per output (one workgroup a window)
    bool counted;             // a single fill takes the counted form
    bool chunk;               // batches take the chunk-speculative form
    double expected_rejections;  // of the launch, as choose_path estimated
    uint32_t chunk_windows;   // its 128-pair windows per chunk (1, 2, 4)
    uint32_t chunk_pairs;     // its pairs per chunk
    uint32_t *zero_word;
    bool spec;
    uint32_t threads;
    uint64_t T;
    prngd_tuning_t tune;
};

prngd_status_t plan_launch(DeviceInfo *d, const Config &cfg, LaunchArgs *args, LaunchPlan *lp,
                           uint32_t default_ppl = 16, bool may_alloc = true)
{
    lp->tune = tuning_for(cfg.fam, cfg.w, default_ppl);
    lp->threads = lp->tune.block_threads;
    // kernels built for Eq. (5) alone, or taking the map's constants
    const uint32_t kfam = cfg.fam | (cfg.map == PRNGD_MAP_EQ5 ? 0u : FAM_ANY_MAP);
    lp->kernel = fill_kernel_for(kfam, lp->threads, lp->tune.pairs_per_lane, false);
    lp->seq_kernel = fill_kernel_for(kfam, lp->threads, lp->tune.pairs_per_lane, true);
    if (!lp->kernel || !lp->seq_kernel)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "no kernel for %u threads x %u pairs per lane",
                    lp->threads, lp->tune.pairs_per_lane);
    if (cfg.arity == 3) {
        // three words per output: the ordered kernels in their one shape
        // (256 threads, 16 triples per thread); no speculative forms
        lp->threads = 256;
        lp->tune.block_threads = 256;
        lp->tune.pairs_per_lane = 16;
        lp->kernel = triple_kernel_for(cfg.fam, false);
        lp->seq_kernel = triple_kernel_for(cfg.fam, true);
        lp->counted_kernels[0] = counted_triple_kernel_for(cfg.fam, false);
        lp->counted_kernels[1] = counted_triple_kernel_for(cfg.fam, true);
        if (!lp->kernel || !lp->seq_kernel)
            return fail(PRNGD_ERR_UNSUPPORTED, "three words per output: no kernel for this "
                                               "generator");
    }
    if (cfg.consume == PRNGD_CONSUME_SINGLE) {
        // one workgroup of 256 threads per segment, windows in order
        const void *k = single_kernel_for(kfam);
        if (!k)
            return fail(PRNGD_ERR_UNSUPPORTED, "single-word consumption needs a single-generator "
                                               "stream (Philox, MRG32k3a or the test generator)");
        lp->threads = 256;
        lp->seq_kernel = k;
        lp->kernel = k;
    }
    lp->T = uint64_t(lp->threads) * lp->tune.pairs_per_lane;
    for (int hold = 0; hold < 2 && cfg.arity == 2; ++hold) {
        lp->spec_kernels[hold][0] = spec_kernel_for(kfam, lp->threads,
                                                    lp->tune.pairs_per_lane, false, false, hold);
        lp->spec_kernels[hold][1] = spec_kernel_for(kfam, lp->threads,
                                                    lp->tune.pairs_per_lane, false, true, hold);
    }
    const bool two = cfg.arity == 2;
    lp->repair_kernel = two ? spec_kernel_for(kfam, lp->threads, lp->tune.pairs_per_lane, true,
                                              false, false)
                            : nullptr;
    lp->spec_kernel = nullptr;
    lp->spec_single_kernel = nullptr;

    lp->words_kernel = two ? spec_words_kernel_for(kfam, false) : nullptr;
    lp->words_repair_kernel = two ? spec_words_kernel_for(kfam, true) : nullptr;
    // the chunk form: a wave takes one chunk of pairs_per_lane / 2 windows
    // (2 pairs per lane each; 1, 2 or 4 windows)
    lp->chunk_windows = std::min<uint32_t>(4, std::max<uint32_t>(1, lp->tune.pairs_per_lane / 2));
    if (lp->chunk_windows == 3)
        lp->chunk_windows = 2;
    lp->chunk_pairs = kChunkPairs * lp->chunk_windows;
    lp->chunk_kernel = two ? chunk_kernel_for(kfam, false, lp->chunk_windows) : nullptr;
    lp->chunk_repair_kernel = two ? chunk_kernel_for(kfam, true, lp->chunk_windows) : nullptr;
    if (two) {
        lp->counted_kernels[0] = counted_kernel_for(kfam, false);
        lp->counted_kernels[1] = counted_kernel_for(kfam, true);
    }
    lp->counted = false;
    lp->counted_triples = false;
    lp->wave_kernel = two ? spec_wave_kernel_for(kfam, false, lp->chunk_windows) : nullptr;
    lp->wave_repair_kernel = two ? spec_wave_kernel_for(kfam, true, lp->chunk_windows) : nullptr;
    lp->wave = false;
    lp->chunk = false;
    lp->expected_rejections = 0.0;
    lp->zero_word = d->zero_word;
    lp->spec = false;                  // decided per launch by choose_path
    args->store_mode = lp->tune.store_mode;
    args->spin_limit = g_spin_limit.load(std::memory_order_relaxed);
    args->w = cfg.w;
    args->a0 = uint32_t(cfg.a0);
    args->a = uint32_t(cfg.a);
    args->b0 = uint32_t(cfg.b0);
    const MapConsts mc = map_consts(cfg);
    args->S = mc.S;
    args->nadd = mc.nadd;
    args->osign = mc.osign;
    args->ooff = mc.ooff;
    args->error = d->error_dev;
    args->mrg_thread = nullptr;
    args->mrg_window = nullptr;
    args->segs = nullptr;
    args->tile_seg = nullptr;
    args->flip = nullptr;
    args->spec = nullptr;
    args->rejlist = nullptr;
    args->hint = nullptr;
    if (cfg.fam == FAM_MRG || cfg.fam == FAM_MIXED) {
        const uint32_t r = cfg.fam == FAM_MRG ? 2u : 1u;
        // one-word consumption steps 16 outputs per thread (8 pairs of 2)
        const uint32_t ppl = cfg.consume == PRNGD_CONSUME_SINGLE ? 8u : lp->tune.pairs_per_lane;
        prngd_status_t st = mrg_tables_for(d, r, ppl, &args->mrg_thread, &args->mrg_window,
                                           may_alloc);
        if (st != PRNGD_OK)
            return st;
    }
    return PRNGD_OK;
}

// Pairs per chunk of the counted single fill (4 windows of 128), and the
// rejections a single fill must expect before it takes that form: with more,
// speculation redoes every chunk in flight when a rejection is published.
// MI355X, 2^22 outputs: w = 24 (0.5 expected) 21 us in 128-pair chunks
// against 25 us counted; w = 20 (8 expected) 52 us against 25 us.  2^28
// outputs: w = 24 881 us against 623 us, w = 17 2781 us ordered against
// 655 us.
constexpr uint64_t kCountedPairs = 512;
constexpr double kCountedMinRejections = 2.0;
// Triples a single fill of three words per output needs to take the counted
// form (four windows of 4096).
constexpr uint64_t kTripleCountedMin = 4 * 4096;

// The longest request (planned pairs) the chunk form takes automatically:
// its repair produces a dirty request again on one wave, about 0.2 us per
// 128-pair window, so a request of 2^16 pairs costs at most about 100 us.
constexpr uint64_t kChunkFormMaxPairs = uint64_t(1) << 16;

// Whether a launch of `pairs` planned pairs whose longest segment has
// `longest` planned pairs takes a speculative fill, and which form.  Automatic
// choice (x1 uniform on [a0, a] rejects 2 / (a - a0 + 1) of the pairs):
// speculation pays when some segment is long enough that ordering its
// tiles across workgroups would cost, and the launch expects few enough
// rejections that the repair pass has little to redo.  Measured on
// MI355X: a batch of requests of at most 2^16 pairs that expects at most
// 256 rejections is fastest in the chunk form (2^16 requests of 2^14
// outputs: 1.56 ms against 1.62 ms ordered).  A single fill of Philox or
// the test generator that expects more than 2 rejections is fastest
// counted; with fewer, at w = 32 in the holding form, at w < 32 in 128-pair
// chunks (w = 24, 2^22 outputs: 21 us against 74 us holding).  Other
// batches take the holding form up to 128 expected rejections; beyond that
// the ordered kernels win.
void choose_path(LaunchPlan *lp, const Config &c, uint64_t pairs, uint64_t longest,
                 bool single, uint64_t nseg = 1)
{
    lp->spec = false;
    lp->wave = false;
    lp->chunk = false;
    lp->counted = false;
    lp->counted_triples = false;
    // three words per output: a single fill of at least kTripleCountedMin
    // triples is counted (path 1 keeps the ordered kernels)
    if (c.arity == 3 && single && lp->tune.path != 1 && lp->counted_kernels[0] &&
        lp->counted_kernels[1] && pairs >= kTripleCountedMin &&
        pairs / lp->T + 2 <= uint64_t(kScanBlock) * kScanBlocksMax) {
        lp->counted = true;
        lp->counted_triples = true;
        return;
    }
    if (!lp->repair_kernel || lp->tune.path == 1 || c.consume == PRNGD_CONSUME_SINGLE)
        return;
    const double rho = 2.0 / double(c.a - c.a0 + 1);
    const double expected = double(pairs) * rho;
    lp->expected_rejections = expected;
    const bool wave_ok = single && lp->wave_kernel && lp->wave_repair_kernel;
    // the chunk form's one-shot grid: 4 chunks per workgroup of 256 threads,
    // at most 2^32 - 1 threads; a segment adds at most one chunk
    const bool chunk_ok = !single && lp->chunk_kernel && lp->chunk_repair_kernel &&
                          pairs / lp->chunk_pairs + nseg < (uint64_t(1) << 26);
    // the counted form's two-level scan: at most kScanBlocksMax blocks of
    // kScanBlock chunks of 512 pairs (a chunk more for the start offset)
    const bool counted_ok = single && lp->counted_kernels[0] && lp->counted_kernels[1] &&
                            pairs / kCountedPairs + 2 <= uint64_t(kScanBlock) * kScanBlocksMax;
    if (counted_ok && (lp->tune.path == 6 ||
                       (lp->tune.path == 0 && longest >= (uint64_t(64) << 12) &&
                        expected > kCountedMinRejections))) {
        lp->counted = true;
        return;
    }
    int hold = -1;
    if (lp->tune.path == 5 && chunk_ok) {
        lp->chunk = true;
        return;
    }
    if (lp->tune.path == 0 && chunk_ok && longest <= kChunkFormMaxPairs && expected <= 256.0) {
        lp->chunk = true;
        return;
    }
    if (lp->tune.path == 4 || lp->tune.path == 5) {
        lp->wave = wave_ok;
        hold = 0;
    } else if (lp->tune.path == 2) {
        hold = 0;
    } else if (lp->tune.path == 3) {
        hold = 1;
    } else if (longest >= (uint64_t(64) << 12)) {
        if (expected <= 2.0 && (c.fam == FAM_PHILOX32 || !wave_ok))
            hold = 1;
        else if (wave_ok && expected <= 1024.0) {
            lp->wave = true;
            hold = 1;
        } else if (expected <= 128.0)
            hold = 1;
    }
    if (hold < 0)
        return;
    // MRG32k3a and mixed have the holding form only
    if (!lp->spec_kernels[hold][0])
        hold = 1;
    lp->spec_kernel = lp->spec_kernels[hold][0];
    lp->spec_single_kernel = lp->spec_kernels[hold][1];
    lp->spec = lp->spec_kernel && lp->spec_single_kernel;
}

// Workgroups of a launch over `units` tiles or segments: all that fit on
// the device at once (or blocks_per_cu per CU), never more than units.
uint32_t grid_for(DeviceInfo *d, const LaunchPlan &lp, const void *kernel, uint64_t units)
{
    const int occ = occupancy_of(d, kernel, lp.threads);
    const uint64_t per_cu = lp.tune.blocks_per_cu ? lp.tune.blocks_per_cu : uint64_t(occ);
    const uint64_t g = std::min<uint64_t>(per_cu * uint64_t(d->cus), units);
    return uint32_t(std::max<uint64_t>(1, g));
}

// Workgroups of a repair launch over `tiles` tiles: each takes a block of
// as many tiles as it has threads per pass.
uint32_t repair_grid(DeviceInfo *d, const LaunchPlan &lp, uint64_t tiles)
{
    const uint64_t blocks = (tiles + lp.threads - 1) / lp.threads;
    return uint32_t(std::max<uint64_t>(1, std::min<uint64_t>(blocks, 2 * uint64_t(d->cus))));
}

// Enqueue the speculative fill of `tiles` tiles and its repair.
prngd_status_t launch_spec(DeviceInfo *d, const LaunchPlan &lp, Workspace *ws, LaunchArgs args,
                           uint64_t tiles, hipStream_t s)
{
    args.spec = ws->spec;
    args.rejlist = ws->rejlist;
    args.hint = ws->hint;
    args.list_cap = uint32_t(std::min<size_t>(ws->spec_cap, 0xFFFFFFFFu));
    args.total_tiles = uint32_t(tiles);
    if (!args.flip)
        args.flip = lp.zero_word;
    HIP_TRY(launch_fill(args.segs ? lp.spec_kernel : lp.spec_single_kernel, uint32_t(tiles),
                        lp.threads, args, s));
    HIP_TRY(launch_fill(lp.repair_kernel, repair_grid(d, lp, tiles), lp.threads, args, s));
    return PRNGD_OK;
}

// Words per window of the one-word-consumption kernels.
constexpr uint64_t kWordsT = 4096;

// Whether a one-word-consumption fill of n outputs takes the speculative
// form across workgroups: automatically from 2^15 outputs while the fill
// expects at most 64 words equal to a0 or a (about 4 n / (a - a0 + 1)),
// when a speculative path is forced while it expects at most 256; the
// segment-sequential kernel otherwise.
bool words_spec_wanted(const LaunchPlan &lp, const Config &c, uint64_t n)
{
    if (!lp.words_kernel || !lp.words_repair_kernel || lp.tune.path == 1)
        return false;
    const double expected = 4.0 * double(n) / double(c.a - c.a0 + 1);
    if (lp.tune.path >= 2)
        return expected <= 256.0;
    return n >= (uint64_t(1) << 15) && expected <= 64.0;
}

// Enqueue the one-word-consumption speculative fill of args.seg0 and its
// repair: one workgroup per window of kWordsT words, one more window than
// the planned words need wherever the start lies in its window.
prngd_status_t launch_spec_words(DeviceInfo *d, const LaunchPlan &lp, Workspace *ws,
                                 LaunchArgs args, hipStream_t s)
{
    const uint64_t words = 2 * args.seg0.planned;
    const uint64_t tiles = (words + kWordsT - 1) / kWordsT + 1;
    if (tiles > kMaxTiles)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "fill too large for the one-word form");
    prngd_status_t st;
    if ((st = ws_prepare_spec(ws, tiles, s)) != PRNGD_OK)
        return st;
    args.spec = ws->spec;
    args.rejlist = ws->rejlist;
    args.hint = ws->hint;
    args.list_cap = uint32_t(std::min<size_t>(ws->spec_cap, 0xFFFFFFFFu));
    args.total_tiles = uint32_t(tiles);
    args.seg0.ntiles = uint32_t(tiles);
    if (!args.flip)
        args.flip = lp.zero_word;
    HIP_TRY(launch_fill(lp.words_kernel, uint32_t(tiles), 256, args, s));
    HIP_TRY(launch_fill(lp.words_repair_kernel, repair_grid(d, lp, tiles), 256, args, s));
    return PRNGD_OK;
}

// Enqueue the wave-granular speculative fill of one segment (args.seg0)
// and its repair: one chunk of lp.chunk_pairs pairs per wave.
prngd_status_t launch_spec_wave(DeviceInfo *d, const LaunchPlan &lp, Workspace *ws,
                                LaunchArgs args, hipStream_t s)
{
    const uint64_t chunks =
        std::max<uint64_t>(1, (args.seg0.planned + lp.chunk_pairs - 1) / lp.chunk_pairs);
    if (chunks > kMaxTiles)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "fill too large for the wave-granular form");
    prngd_status_t st;
    if ((st = ws_prepare_spec(ws, chunks, s)) != PRNGD_OK)
        return st;
    if ((st = ws_prepare_hint64(ws, chunks, s)) != PRNGD_OK)
        return st;
    args.spec = ws->spec;
    args.rejlist = ws->rejlist;
    args.hint = ws->hint;
    args.hint64 = ws->hint64;
    args.epoch = ++ws->spec_epoch;
    args.total_tiles = uint32_t(chunks);
    if (!args.flip)
        args.flip = lp.zero_word;
    // one-shot grid: a workgroup covers 4 waves of one chunk each
    const uint64_t grid = (chunks + 3) / 4;
    if (grid > 0xFFFFFFFFull)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "fill too large for the wave-granular form");
    HIP_TRY(launch_fill(lp.wave_kernel, uint32_t(grid), 256, args, s));
    const uint32_t rgrid = uint32_t(
        std::max<uint64_t>(1, std::min<uint64_t>((chunks + 255) / 256, 2 * uint64_t(d->cus))));
    HIP_TRY(launch_fill(lp.wave_repair_kernel, rgrid, 256, args, s));
    return PRNGD_OK;
}

// Workgroups (of 16 waves) of the chunk form's repair: each takes dirty
// segments b, b + G, ...; the launch never knows how many there are.
constexpr uint32_t kChunkRepairThreads = 1024;

uint32_t chunk_repair_grid(DeviceInfo *d, uint64_t nseg, double expected)
{
    // sized to the dirty requests expected (a launch of idle workgroups
    // costs), at least 8, at most two per CU
    const double want = std::max(8.0, std::ceil(4.0 * expected));
    const uint64_t g = std::min<uint64_t>(2 * uint64_t(d->cus), uint64_t(want));
    return uint32_t(std::max<uint64_t>(1, std::min<uint64_t>(nseg, g)));
}

// Workgroups of the chunk form's one-shot grid over `chunks` chunks: 4
// waves of one chunk each.
uint32_t chunk_grid(uint64_t chunks)
{
    return uint32_t((chunks + 3) / 4);
}

// Kernel arguments of the chunk-speculative fill of args.nseg segments in
// args.total_tiles chunks; chunks_per_seg (if nonzero) with the constants
// of the division by it (multiply-high, add, shift: Granlund and
// Montgomery's round-up method, exact for every 32-bit dividend).
LaunchArgs chunk_args(const LaunchPlan &lp, Workspace *ws, LaunchArgs args,
                      uint32_t chunks_per_seg)
{
    args.spec = ws->spec;
    args.chunk_segs = ws->chunk_segs;
    args.first_dirty = ws->first_dirty;
    args.dirty_list = ws->dirty_list;
    args.chunks_per_seg = chunks_per_seg;
    args.cps_magic = 0;
    args.cps_shift = 0;
    if (chunks_per_seg >= 2) {
        uint32_t l = 0;
        while ((uint64_t(1) << l) < chunks_per_seg)
            ++l;
        const uint64_t num = (uint64_t(1) << 32) * ((uint64_t(1) << l) - chunks_per_seg);
        args.cps_magic = uint32_t(num / chunks_per_seg + 1);
        args.cps_shift = l - 1;
    }
    args.chunk_shift = 0;
    while ((uint32_t(1) << args.chunk_shift) < lp.chunk_pairs)
        ++args.chunk_shift;
    if (!args.flip)
        args.flip = lp.zero_word;
    return args;
}

// Enqueue the chunk-speculative fill of a batch: the segments' records for
// this launch, the one-shot grid of chunks (4 per workgroup), the repair.
prngd_status_t launch_chunk(DeviceInfo *d, const LaunchPlan &lp, Workspace *ws,
                            const LaunchArgs &in, uint32_t chunks_per_seg, hipStream_t s)
{
    const LaunchArgs args = chunk_args(lp, ws, in, chunks_per_seg);
    HIP_TRY(launch_fill(chunk_prep_kernel_ptr(), (args.nseg + 255) / 256, 256, args, s));
    HIP_TRY(launch_fill(lp.chunk_kernel, chunk_grid(args.total_tiles), 256, args, s));
    HIP_TRY(launch_fill(lp.chunk_repair_kernel,
                        chunk_repair_grid(d, args.nseg, lp.expected_rejections),
                        kChunkRepairThreads, args, s));
    return PRNGD_OK;
}

// Enqueue the counted fill of one segment (args.seg0): count every chunk,
// scan the counts in two levels, produce every chunk at its offset.
prngd_status_t launch_counted(const LaunchPlan &lp, Workspace *ws, LaunchArgs args,
                              hipStream_t s)
{
    // pairs per chunk of one wave, or triples per window of one workgroup
    const uint64_t unit = lp.counted_triples ? lp.T : kCountedPairs;
    const uint64_t chunks = std::max<uint64_t>(1, (args.seg0.planned + unit - 1) / unit);
    if (chunks > uint64_t(kScanBlock) * kScanBlocksMax)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "fill too large for the counted form");
    prngd_status_t st;
    if ((st = ws_prepare_counted(ws, chunks)) != PRNGD_OK)
        return st;
    args.chunk_counts = ws->counts;
    args.chunk_offs = ws->count_offs;
    args.block_offs = ws->block_offs;
    args.total_tiles = uint32_t(chunks);
    if (!args.flip)
        args.flip = lp.zero_word;
    const uint32_t grid = uint32_t(lp.counted_triples ? chunks : (chunks + 3) / 4);
    const uint32_t nblocks = uint32_t((chunks + kScanBlock - 1) / kScanBlock);
    HIP_TRY(launch_fill(lp.counted_kernels[0], grid, 256, args, s));
    HIP_TRY(launch_fill(counted_scan_kernel_ptr(false), nblocks, 1024, args, s));
    HIP_TRY(launch_fill(counted_scan_kernel_ptr(true), 1, 1024, args, s));
    HIP_TRY(launch_fill(lp.counted_kernels[1], grid, 256, args, s));
    return PRNGD_OK;
}

// Fill the descriptor of one request; returns its number of tiles.
prngd_status_t make_segment(prngd_handle_t h, uint64_t n, double *out, uint64_t T,
                            uint32_t slack_mode, uint64_t tile_begin, Segment *s,
                            uint64_t *ntiles)
{
    if (n > kMaxOutputs)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "n = %llu exceeds 2^38 - 1 outputs per fill",
                    (unsigned long long)n);
    if (!out || (reinterpret_cast<uintptr_t>(out) & 7u))
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "out must be a non-null 8-byte aligned pointer");
    const uint64_t planned = planned_pairs(h->cfg, n, slack_mode);
    const uint64_t tiles = std::max<uint64_t>(1, (planned + T - 1) / T);
    if (tile_begin + tiles > kMaxTiles)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "launch too large (more than 2^31 tiles)");
    s->seed = h->seed;
    s->n = n;
    s->planned = planned;
    s->out = out;
    s->counter = h->slot;
    s->stream_id = h->stream_id;
    s->parity = h->parity;
    s->tile_begin = uint32_t(tile_begin);
    s->ntiles = uint32_t(tiles);
    std::memcpy(s->mrg, h->mrg, sizeof s->mrg);
    *ntiles = tiles;
    return PRNGD_OK;
}

bool same_config(const Config &x, const Config &y)
{
    return x.fam == y.fam && x.w == y.w && x.a0 == y.a0 && x.a == y.a && x.b0 == y.b0 &&
           x.b == y.b && x.map == y.map && x.consume == y.consume && x.arity == y.arity;
}

// The MRG32k3a jump tables the look-back kernel of a handle with this
// configuration takes in its current launch shape, built when the handle
// is created (so that prngd_fill_noalloc finds them).
prngd_status_t default_mrg_tables(DeviceInfo *d, const Config &cfg)
{
    const uint32_t r = cfg.fam == FAM_MRG ? 2u : 1u;
    const uint32_t ppl = tuning_for(cfg.fam, cfg.w).pairs_per_lane;
    const uint32_t *t = nullptr, *w = nullptr;
    return mrg_tables_for(d, r, ppl, &t, &w);
}

prngd_status_t current_device(int *dev)
{
    HIP_TRY(hipGetDevice(dev));
    return PRNGD_OK;
}

// A validated request list split for the two kernels: `lb` segments (with
// tile_begin set, tiles in order) for the look-back kernel, `seq` segments
// (largest first) for the segment-sequential kernel.
struct BatchPlan {
    std::vector<Segment> lb;
    std::vector<Segment> seq;
    std::vector<prngd_handle_t> handles;
    uint64_t lb_tiles = 0;
    uint32_t chunks_per_seg = 0;   // chunk form: every segment's chunk count, if equal and >= 2
};

prngd_status_t build_batch(DeviceInfo *d, LaunchPlan &lp, const prngd_request_t *reqs,
                           uint32_t count, BatchPlan *bp)
{
    if (!reqs || count == 0)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "empty request list");
    std::unordered_set<prngd_handle_t> seen;
    const prngd_handle_t first = reqs[0].h;
    if (!first)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "request 0 has a NULL handle");
    // validate, and plan the pairs that decide the path
    uint64_t pairs = 0, max_seg_pairs = 0, live = 0;
    for (uint32_t i = 0; i < count; ++i) {
        const prngd_request_t &r = reqs[i];
        if (!r.h)
            return fail(PRNGD_ERR_INVALID_ARGUMENT, "request %u has a NULL handle", i);
        if (!seen.insert(r.h).second)
            return fail(PRNGD_ERR_INVALID_ARGUMENT, "handle of request %u repeats", i);
        if (!same_config(r.h->cfg, first->cfg) || r.h->device != first->device)
            return fail(PRNGD_ERR_INVALID_ARGUMENT,
                        "request %u: all handles of a batch must share generator, k, min, max",
                        i);
        if (r.h->plan)
            return fail(PRNGD_ERR_INVALID_ARGUMENT, "request %u: handle bound to a plan", i);
        if (r.n == 0 || r.n > kMaxOutputs)
            continue;
        const uint64_t planned = planned_pairs(r.h->cfg, r.n, lp.tune.slack_mode);
        pairs += planned;
        max_seg_pairs = std::max<uint64_t>(max_seg_pairs, planned);
        ++live;
    }
    choose_path(&lp, first->cfg, pairs, max_seg_pairs, false, live);
    // the chunk form plans its segments in chunks, the others in tiles
    const uint64_t T = lp.chunk ? lp.chunk_pairs : lp.T;
    std::vector<Segment> all;
    uint64_t total = 0;
    for (uint32_t i = 0; i < count; ++i) {
        const prngd_request_t &r = reqs[i];
        if (r.n == 0)
            continue;
        Segment s;
        uint64_t nt = 0;
        prngd_status_t st = make_segment(r.h, r.n, r.out, T, lp.tune.slack_mode, 0, &s, &nt);
        if (st != PRNGD_OK)
            return st;
        total += nt;
        all.push_back(s);
        bp->handles.push_back(r.h);
    }
    const uint64_t wg = uint64_t(occupancy_of(d, lp.seq_kernel, lp.threads)) * uint64_t(d->cus);
    // the speculative fills take every segment tile by tile; single-word
    // consumption every segment whole
    const uint64_t limit = first->cfg.consume == PRNGD_CONSUME_SINGLE
                               ? ~uint64_t(0)
                               : lp.spec || lp.chunk ? 0 : seq_limit(lp.tune, total, wg);
    for (const Segment &s : all) {
        if (s.ntiles <= limit) {
            bp->seq.push_back(s);
        } else {
            Segment t = s;
            if (bp->lb_tiles + t.ntiles > kMaxTiles)
                return fail(PRNGD_ERR_INVALID_ARGUMENT, "launch too large (more than 2^32 tiles)");
            t.tile_begin = uint32_t(bp->lb_tiles);
            bp->lb_tiles += t.ntiles;
            bp->lb.push_back(t);
        }
    }
    std::stable_sort(bp->seq.begin(), bp->seq.end(),
                     [](const Segment &x, const Segment &y) { return x.ntiles > y.ntiles; });
    // segments of equal length (two chunks or more) find theirs by a division
    bp->chunks_per_seg = 0;
    if (lp.chunk && !bp->lb.empty() && bp->lb[0].ntiles >= 2 &&
        std::all_of(bp->lb.begin(), bp->lb.end(),
                    [&](const Segment &x) { return x.ntiles == bp->lb[0].ntiles; }))
        bp->chunks_per_seg = bp->lb[0].ntiles;
    return PRNGD_OK;
}

}  // namespace

// ================================================================= C ABI
extern "C" {

const char *prngd_status_string(prngd_status_t s)
{
    switch (s) {
    case PRNGD_OK: return "PRNGD_OK";
    case PRNGD_ERR_INVALID_ARGUMENT: return "PRNGD_ERR_INVALID_ARGUMENT";
    case PRNGD_ERR_UNSUPPORTED: return "PRNGD_ERR_UNSUPPORTED";
    case PRNGD_ERR_OUT_OF_MEMORY: return "PRNGD_ERR_OUT_OF_MEMORY";
    case PRNGD_ERR_HIP: return "PRNGD_ERR_HIP";
    case PRNGD_ERR_DEVICE: return "PRNGD_ERR_DEVICE";
    }
    return "PRNGD_ERR_UNKNOWN";
}

const char *prngd_last_error(void)
{
    return g_last_error.c_str();
}

prngd_status_t prngd_describe(prngd_generator_t generator, double k, uint64_t min, uint64_t max,
                              uint32_t *w, uint64_t *b0, uint64_t *b, uint64_t *D, double *S)
{
    Config c;
    prngd_status_t st = make_config(generator, k, min, max, &c);
    if (st != PRNGD_OK)
        return st;
    if (w) *w = c.w;
    if (b0) *b0 = c.b0;
    if (b) *b = c.b;
    if (D) *D = c.D;
    if (S) *S = c.S;
    return PRNGD_OK;
}

prngd_status_t prngd_describe_map(prngd_generator_t generator, double k, uint64_t min,
                                  uint64_t max, prngd_map_t map, uint64_t *n_offset,
                                  uint64_t *D, double *S)
{
    Config c;
    prngd_status_t st = make_config(generator, k, min, max, &c);
    if (st != PRNGD_OK)
        return st;
    if (map != PRNGD_MAP_EQ5 && map != PRNGD_MAP_EQ4 && map != PRNGD_MAP_ONE_MINUS)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "unknown map %d", int(map));
    c.map = uint32_t(map);
    if (n_offset)
        *n_offset = map == PRNGD_MAP_EQ4 ? (uint64_t(1) << c.w) - (c.b - c.b0) : 0;
    if (D)
        *D = map == PRNGD_MAP_EQ4 ? c.D4 : c.D;
    if (S)
        *S = map == PRNGD_MAP_EQ4 ? c.S4 : c.S;
    return PRNGD_OK;
}

prngd_status_t prngd_set_map(prngd_handle_t h, prngd_map_t map)
{
    if (!h)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "NULL handle");
    if (map != PRNGD_MAP_EQ5 && map != PRNGD_MAP_EQ4 && map != PRNGD_MAP_ONE_MINUS)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "unknown map %d", int(map));
    std::lock_guard<std::recursive_mutex> lock(g_mutex);
    if (h->plan)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "handle is bound to a live plan");
    if (map != PRNGD_MAP_EQ5 && h->cfg.arity == 3)
        return fail(PRNGD_ERR_UNSUPPORTED, "three words per output take Eq. (5)");
    h->cfg.map = uint32_t(map);
    return PRNGD_OK;
}

prngd_status_t prngd_set_consume(prngd_handle_t h, prngd_consume_t consume)
{
    if (!h)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "NULL handle");
    if (consume != PRNGD_CONSUME_PAIR && consume != PRNGD_CONSUME_SINGLE)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "unknown consumption mode %d", int(consume));
    std::lock_guard<std::recursive_mutex> lock(g_mutex);
    if (h->plan)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "handle is bound to a live plan");
    if (consume != PRNGD_CONSUME_PAIR && h->cfg.arity == 3)
        return fail(PRNGD_ERR_UNSUPPORTED, "three words per output take pair consumption");
    if (consume == PRNGD_CONSUME_SINGLE && !single_kernel_for(h->cfg.fam))
        return fail(PRNGD_ERR_UNSUPPORTED,
                    "single-word consumption needs a single-generator stream (Philox, MRG32k3a "
                    "or the test generator)");
    h->cfg.consume = uint32_t(consume);
    return PRNGD_OK;
}

prngd_status_t prngd_set_arity(prngd_handle_t h, uint32_t words)
{
    if (!h)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "NULL handle");
    if (words != 2 && words != 3)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "words per output must be 2 or 3, not %u", words);
    std::lock_guard<std::recursive_mutex> lock(g_mutex);
    if (h->plan)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "handle is bound to a live plan");
    if (words == 3) {
        if (!triple_kernel_for(h->cfg.fam, false))
            return fail(PRNGD_ERR_UNSUPPORTED, "three words per output: Philox4x32-10 and the "
                                               "test generator only");
        if (h->cfg.map != PRNGD_MAP_EQ5 || h->cfg.consume != PRNGD_CONSUME_PAIR)
            return fail(PRNGD_ERR_UNSUPPORTED, "three words per output take Eq. (5) and pair "
                                               "consumption");
        h->cfg.S3 = folded_constant3(h->cfg.w, triple_denominator(h->cfg));
    }
    h->cfg.arity = words;
    return PRNGD_OK;
}

prngd_status_t prngd_get_arity(prngd_handle_t h, uint32_t *words)
{
    if (!h || !words)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "NULL argument");
    *words = h->cfg.arity;
    return PRNGD_OK;
}

prngd_status_t prngd_get_consume(prngd_handle_t h, prngd_consume_t *consume)
{
    if (!h || !consume)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "NULL argument");
    *consume = static_cast<prngd_consume_t>(h->cfg.consume);
    return PRNGD_OK;
}

prngd_status_t prngd_get_map(prngd_handle_t h, prngd_map_t *map)
{
    if (!h || !map)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "NULL argument");
    *map = static_cast<prngd_map_t>(h->cfg.map);
    return PRNGD_OK;
}

prngd_status_t prngd_create(uint64_t seed, prngd_generator_t generator, double k, uint64_t min,
                            uint64_t max, prngd_handle_t *out_handle)
{
    if (!out_handle)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "out_handle is NULL");
    *out_handle = nullptr;
    Config cfg;
    prngd_status_t st = make_config(generator, k, min, max, &cfg);
    if (st != PRNGD_OK)
        return st;
    std::lock_guard<std::recursive_mutex> lock(g_mutex);
    int dev = 0;
    if ((st = current_device(&dev)) != PRNGD_OK)
        return st;
    DeviceInfo *d = nullptr;
    if ((st = device_info(dev, &d)) != PRNGD_OK)
        return st;
    std::unique_ptr<prngd_handle_s> h(new prngd_handle_s);
    h->device = dev;
    h->gen = generator;
    h->cfg = cfg;
    h->seed = seed;
    if (cfg.fam == FAM_MRG || cfg.fam == FAM_MIXED) {
        mrg_stream_base(seed, 0, h->mrg);
        if ((st = default_mrg_tables(d, cfg)) != PRNGD_OK)
            return st;
    }
    if ((st = alloc_slot(d, &h->slot)) != PRNGD_OK)
        return st;
    if (cfg.fam == FAM_RANMAR) {
        if ((st = alloc_ranmar(d, &h->rm)) != PRNGD_OK ||
            (st = ranmar_init_states({{h->rm, nullptr}}, seed, 0)) != PRNGD_OK) {
            d->free_slots.push_back(h->slot);
            if (h->rm)
                d->rm_free.push_back(h->rm);
            return st;
        }
    }
    *out_handle = h.release();
    return PRNGD_OK;
}

prngd_status_t prngd_create_many(uint64_t seed, prngd_generator_t generator, double k,
                                 uint64_t min, uint64_t max, uint32_t first_stream_id,
                                 uint32_t count, prngd_handle_t *handles)
{
    if (!handles)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "handles is NULL");
    if (count && uint64_t(first_stream_id) + count - 1 > 0xFFFFFFFFull)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "substream ids beyond 2^32 - 1");
    Config cfg;
    prngd_status_t st = make_config(generator, k, min, max, &cfg);
    if (st != PRNGD_OK)
        return st;
    std::lock_guard<std::recursive_mutex> lock(g_mutex);
    int dev = 0;
    if ((st = current_device(&dev)) != PRNGD_OK)
        return st;
    DeviceInfo *d = nullptr;
    if ((st = device_info(dev, &d)) != PRNGD_OK)
        return st;
    if ((cfg.fam == FAM_MRG || cfg.fam == FAM_MIXED) &&
        (st = default_mrg_tables(d, cfg)) != PRNGD_OK)
        return st;
    for (uint32_t i = 0; i < count; ++i) {
        std::unique_ptr<prngd_handle_s> h(new prngd_handle_s);
        h->device = dev;
        h->gen = generator;
        h->cfg = cfg;
        h->seed = seed;
        h->stream_id = first_stream_id + i;
        if (cfg.fam == FAM_MRG || cfg.fam == FAM_MIXED)
            mrg_stream_base(seed, h->stream_id, h->mrg);
        if ((st = alloc_slot(d, &h->slot)) != PRNGD_OK) {
            for (uint32_t j = 0; j < i; ++j) {
                d->free_slots.push_back(handles[j]->slot);
                delete handles[j];
                handles[j] = nullptr;
            }
            return st;
        }
        handles[i] = h.release();
    }
    if (cfg.fam == FAM_RANMAR && count) {
        std::vector<std::pair<RanmarState *, const void *>> hs;
        for (uint32_t i = 0; i < count && st == PRNGD_OK; ++i) {
            st = alloc_ranmar(d, &handles[i]->rm);
            hs.push_back({handles[i]->rm, nullptr});
        }
        if (st == PRNGD_OK)
            st = ranmar_init_states(hs, seed, first_stream_id);
        if (st != PRNGD_OK) {
            for (uint32_t i = 0; i < count; ++i) {
                d->free_slots.push_back(handles[i]->slot);
                if (handles[i]->rm)
                    d->rm_free.push_back(handles[i]->rm);
                delete handles[i];
                handles[i] = nullptr;
            }
            return st;
        }
    }
    return PRNGD_OK;
}

prngd_status_t prngd_destroy(prngd_handle_t h)
{
    if (!h)
        return PRNGD_OK;
    std::lock_guard<std::recursive_mutex> lock(g_mutex);
    if (h->plan)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "handle is bound to a live plan");
    if (h->last_event)
        HIP_TRY(hipEventSynchronize(h->last_event));
    auto it = g_devices.find(h->device);
    if (it != g_devices.end()) {
        it->second.free_slots.push_back(h->slot);
        if (h->rm)
            it->second.rm_free.push_back(h->rm);
    }
    delete h;
    return PRNGD_OK;
}

int prngd_probe_set_spin_limit(uint32_t polls)
{
    g_spin_limit.store(polls, std::memory_order_relaxed);
    return 0;
}

prngd_status_t prngd_ranmar_state(uint64_t seed, uint32_t stream_id, uint64_t pair_counter,
                                  uint32_t out[98])
{
    if (!out)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "out is NULL");
    uint32_t w[kRanmarRow];
    const unsigned __int128 word = static_cast<unsigned __int128>(pair_counter) * 2u;
    ranmar_window_at(seed, stream_id, uint64_t(word), uint64_t(word >> 64), w);
    std::memcpy(out, w, 98 * sizeof(uint32_t));
    return PRNGD_OK;
}

prngd_status_t prngd_set_position(prngd_handle_t h, uint32_t stream_id, uint64_t pair_counter,
                                  void *stream)
{
    if (!h)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "NULL handle");
    if (h->plan)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "handle is bound to a live plan");
    std::lock_guard<std::recursive_mutex> lock(g_mutex);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace *ws = nullptr;
    prngd_status_t st = stream_workspace(h->device, s, &ws);
    if (st != PRNGD_OK)
        return st;
    if ((st = order_after(h, s)) != PRNGD_OK)
        return st;
    h->stream_id = stream_id;
    if (h->cfg.fam == FAM_MRG || h->cfg.fam == FAM_MIXED)
        mrg_stream_base(h->seed, stream_id, h->mrg);
    if (h->cfg.fam == FAM_RANMAR) {
        // the window at word 2 pair_counter of the stream, both slots
        RanmarInit r{};
        r.dst = h->rm;
        r.slot = h->slot;
        r.counter = pair_counter;
        const unsigned __int128 word = static_cast<unsigned __int128>(pair_counter) * 2u;
        ranmar_window_at(h->seed, stream_id, uint64_t(word), uint64_t(word >> 64), r.words);
        HIP_TRY(launch_ranmar_set(r, s));
    } else {
        HIP_TRY(launch_set_counter(h->slot, pair_counter, s));
    }
    HIP_TRY(hipEventRecord(ws->last, s));
    h->last_event = ws->last;
    h->last_stream = s;
    return PRNGD_OK;
}

prngd_status_t prngd_get_position(prngd_handle_t h, uint32_t *stream_id, uint64_t *pair_counter,
                                  void *stream)
{
    if (!h)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "NULL handle");
    std::lock_guard<std::recursive_mutex> lock(g_mutex);
    hipStream_t s = static_cast<hipStream_t>(stream);
    prngd_status_t st = order_after(h, s);
    if (st != PRNGD_OK)
        return st;
    uint32_t parity = h->parity;
    if (h->plan) {
        // position after the plan's launches so far
        const prngd_plan_s *p = h->plan;
        parity = p->base_parity[h->plan_index] ^ uint32_t(p->launches & 1u);
    }
    uint64_t value = 0;
    HIP_TRY(hipMemcpyAsync(&value, h->slot + parity, sizeof value, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (stream_id)
        *stream_id = h->stream_id;
    if (pair_counter)
        *pair_counter = value;
    return PRNGD_OK;
}

static prngd_status_t fill_batch_impl(const prngd_request_t *reqs, uint32_t count,
                                      void *stream);

// ------------------------------------------------------------------ RANMAR
// Pairs of a segment of a long RANMAR fill (one wave each): fine segments
// while a fill needs at most kRanmarFineSegs of them (more waves for fills
// of up to 2^22 pairs), coarse ones beyond (each wave's jump is then a
// smaller share of its work, and the table stays small).  Requests of a
// batch up to kRanmarWaveMax planned pairs take one wave each; longer ones
// are filled one by one in segments.
constexpr uint32_t kRanmarSegPairs[2] = {1024, 8192};
constexpr uint64_t kRanmarFineSegs = 4096;
constexpr uint64_t kRanmarWaveMax = 32768;

// Rows [0, rows) of jump table `which` on the device; new rows are computed
// on the host (one polynomial product each) and the table is copied whole.
static prngd_status_t ranmar_jump_table(DeviceInfo *d, int which, uint32_t rows)
{
    if (rows <= d->rm_jump_rows[which])
        return PRNGD_OK;
    std::vector<uint32_t> &host = d->rm_jump_host[which];
    const uint32_t have = uint32_t(host.size() / kRanmarRow);
    const uint32_t cap = std::max<uint32_t>({rows, 2 * have, 256u});
    host.resize(size_t(cap) * kRanmarRow);
    ranmar_jump_rows(kRanmarSegPairs[which], have, cap - have,
                     host.data() + size_t(have) * kRanmarRow);
    void *p = nullptr;
    HIP_TRY(hipMalloc(&p, host.size() * sizeof(uint32_t)));
    HIP_TRY(hipMemcpy(p, host.data(), host.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    if (d->rm_jump[which]) {
        HIP_TRY(hipDeviceSynchronize());       // no launch reads the old table any more
        HIP_TRY(hipFree(d->rm_jump[which]));
    }
    d->rm_jump[which] = static_cast<uint32_t *>(p);
    d->rm_jump_rows[which] = cap;
    return PRNGD_OK;
}

static LaunchArgs ranmar_args(DeviceInfo *d, const Config &c)
{
    LaunchArgs a{};
    a.store_mode = 0;
    a.w = c.w;
    a.a0 = uint32_t(c.a0);
    a.a = uint32_t(c.a);
    a.b0 = uint32_t(c.b0);
    const MapConsts mc = map_consts(c);
    a.S = mc.S;
    a.nadd = mc.nadd;
    a.osign = mc.osign;
    a.ooff = mc.ooff;
    a.flip = d->zero_word;
    a.error = d->error_dev;
    a.ranmar_seg_pairs = kRanmarSegPairs[0];
    return a;
}

static uint32_t ranmar_kfam(const Config &c)
{
    return FAM_RANMAR | (c.map == PRNGD_MAP_EQ5 ? 0u : FAM_ANY_MAP);
}

// Enqueue the fill of one RANMAR handle: one wave if it plans at most one
// segment; else count every segment's accepted pairs, scan, produce.
static prngd_status_t ranmar_fill(DeviceInfo *d, prngd_handle_t h, uint64_t n, double *out,
                                  Workspace *ws, hipStream_t s)
{
    Segment seg{};
    uint64_t ntiles = 0;
    prngd_status_t st = make_segment(h, n, out, kRanmarSegPairs[0], 0, 0, &seg, &ntiles);
    if (st != PRNGD_OK)
        return st;
    seg.seed = reinterpret_cast<uint64_t>(h->rm);
    const int which = ntiles <= kRanmarFineSegs ? 0 : 1;
    const uint64_t P = kRanmarSegPairs[which];
    const uint64_t segs = std::max<uint64_t>(1, (seg.planned + P - 1) / P);
    if (segs > uint64_t(kScanBlock) * kScanBlocksMax)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "n = %llu: too large for one RANMAR fill",
                    (unsigned long long)n);
    LaunchArgs a = ranmar_args(d, h->cfg);
    a.seg0 = seg;
    a.nseg = 1;
    a.ranmar_seg_pairs = uint32_t(P);
    const uint32_t kfam = ranmar_kfam(h->cfg);
    if (segs == 1) {
        a.total_tiles = 1;
        HIP_TRY(launch_fill(ranmar_kernel_for(kfam, 0), 1, 256, a, s));
        return PRNGD_OK;
    }
    if ((st = ranmar_jump_table(d, which, uint32_t(segs))) != PRNGD_OK)
        return st;
    if ((st = ws_prepare_counted(ws, segs)) != PRNGD_OK)
        return st;
    a.ranmar_jump = d->rm_jump[which];
    a.chunk_counts = ws->counts;
    a.chunk_offs = ws->count_offs;
    a.block_offs = ws->block_offs;
    a.total_tiles = uint32_t(segs);
    const uint32_t grid = uint32_t((segs + 3) / 4);
    const uint32_t nblocks = uint32_t((segs + kScanBlock - 1) / kScanBlock);
    HIP_TRY(launch_fill(ranmar_kernel_for(kfam, 1), grid, 256, a, s));
    HIP_TRY(launch_fill(counted_scan_kernel_ptr(false), nblocks, 1024, a, s));
    HIP_TRY(launch_fill(counted_scan_kernel_ptr(true), 1, 1024, a, s));
    HIP_TRY(launch_fill(ranmar_kernel_for(kfam, 2), grid, 256, a, s));
    return PRNGD_OK;
}

// A batch of RANMAR requests: short ones one wave each in one launch, long
// ones as single fills, all on `s`.
static prngd_status_t ranmar_batch(DeviceInfo *d, const prngd_request_t *reqs, uint32_t count,
                                   hipStream_t s)
{
    std::unordered_set<prngd_handle_t> seen;
    const prngd_handle_t first = reqs[0].h;
    for (uint32_t i = 0; i < count; ++i) {
        const prngd_request_t &r = reqs[i];
        if (!r.h)
            return fail(PRNGD_ERR_INVALID_ARGUMENT, "request %u has a NULL handle", i);
        if (!seen.insert(r.h).second)
            return fail(PRNGD_ERR_INVALID_ARGUMENT, "handle of request %u repeats", i);
        if (!same_config(r.h->cfg, first->cfg) || r.h->device != first->device)
            return fail(PRNGD_ERR_INVALID_ARGUMENT,
                        "request %u: all handles of a batch must share generator, k, min, max",
                        i);
        if (r.h->plan)
            return fail(PRNGD_ERR_INVALID_ARGUMENT, "request %u: handle bound to a plan", i);
        if (r.n > kMaxOutputs)
            return fail(PRNGD_ERR_INVALID_ARGUMENT, "request %u: n exceeds 2^38 - 1 outputs", i);
        if (r.n && (!r.out || (reinterpret_cast<uintptr_t>(r.out) & 7u)))
            return fail(PRNGD_ERR_INVALID_ARGUMENT,
                        "request %u: out must be a non-null 8-byte aligned pointer", i);
    }
    Workspace *ws = nullptr;
    prngd_status_t st = stream_workspace(first->device, s, &ws);
    if (st != PRNGD_OK)
        return st;
    std::unordered_set<hipEvent_t> waited;
    for (uint32_t i = 0; i < count; ++i) {
        const prngd_handle_t h = reqs[i].h;
        if (reqs[i].n && h->last_event && h->last_stream != s && waited.insert(h->last_event).second)
            HIP_TRY(hipStreamWaitEvent(s, h->last_event, 0));
    }
    std::vector<Segment> segs;
    for (uint32_t i = 0; i < count; ++i) {
        const prngd_request_t &r = reqs[i];
        if (r.n == 0)
            continue;
        if (planned_pairs(r.h->cfg, r.n, 0) > kRanmarWaveMax) {
            if ((st = ranmar_fill(d, r.h, r.n, r.out, ws, s)) != PRNGD_OK)
                return st;
            continue;
        }
        Segment seg{};
        uint64_t ntiles = 0;
        if ((st = make_segment(r.h, r.n, r.out, kRanmarSegPairs[0], 0, 0, &seg, &ntiles)) != PRNGD_OK)
            return st;
        seg.seed = reinterpret_cast<uint64_t>(r.h->rm);
        segs.push_back(seg);
    }
    if (!segs.empty()) {
        const size_t nseg = segs.size();
        if ((st = ws_grow(ws, &ws->dsegs, &ws->dsegs_cap, nseg, s)) != PRNGD_OK)
            return st;
        const int slot = ws->hcur;
        ws->hcur ^= 1;
        HIP_TRY(hipEventSynchronize(ws->hsegs_done[slot]));
        if (ws->hsegs_cap[slot] < nseg) {
            if (ws->hsegs[slot])
                ws->retired_host.push_back(ws->hsegs[slot]);
            void *p = nullptr;
            const size_t cap = std::max<size_t>({nseg, size_t(1024), 2 * ws->hsegs_cap[slot]});
            HIP_TRY(hipHostMalloc(&p, cap * sizeof(Segment), hipHostMallocDefault));
            ws->hsegs[slot] = static_cast<Segment *>(p);
            ws->hsegs_cap[slot] = cap;
        }
        std::copy(segs.begin(), segs.end(), ws->hsegs[slot]);
        HIP_TRY(hipMemcpyAsync(ws->dsegs, ws->hsegs[slot], nseg * sizeof(Segment),
                               hipMemcpyHostToDevice, s));
        HIP_TRY(hipEventRecord(ws->hsegs_done[slot], s));
        LaunchArgs a = ranmar_args(d, first->cfg);
        a.segs = ws->dsegs;
        a.nseg = uint32_t(nseg);
        a.total_tiles = uint32_t(nseg);
        HIP_TRY(launch_fill(ranmar_kernel_for(ranmar_kfam(first->cfg), 0),
                            uint32_t((nseg + 3) / 4), 256, a, s));
    }
    HIP_TRY(hipEventRecord(ws->last, s));
    for (uint32_t i = 0; i < count; ++i) {
        const prngd_handle_t h = reqs[i].h;
        if (reqs[i].n == 0)
            continue;
        h->parity ^= 1u;
        h->last_event = ws->last;
        h->last_stream = s;
    }
    return PRNGD_OK;
}

// A resident batch of RANMAR requests: one wave per request (each of at
// most kRanmarWaveMax planned pairs), then the replay-parity toggle, in a
// HIP graph.
static prngd_status_t ranmar_plan_create(DeviceInfo *d, const prngd_request_t *reqs,
                                         uint32_t count, prngd_plan_t *out_plan)
{
    std::unordered_set<prngd_handle_t> seen;
    const prngd_handle_t first = reqs[0].h;
    std::vector<Segment> segs;
    std::unique_ptr<prngd_plan_s> p(new prngd_plan_s);
    p->device = first->device;
    for (uint32_t i = 0; i < count; ++i) {
        const prngd_request_t &r = reqs[i];
        if (!r.h)
            return fail(PRNGD_ERR_INVALID_ARGUMENT, "request %u has a NULL handle", i);
        if (!seen.insert(r.h).second)
            return fail(PRNGD_ERR_INVALID_ARGUMENT, "handle of request %u repeats", i);
        if (!same_config(r.h->cfg, first->cfg) || r.h->device != first->device)
            return fail(PRNGD_ERR_INVALID_ARGUMENT,
                        "request %u: all handles of a batch must share generator, k, min, max",
                        i);
        if (r.h->plan)
            return fail(PRNGD_ERR_INVALID_ARGUMENT, "request %u: handle bound to a plan", i);
        if (r.n == 0)
            continue;
        if (planned_pairs(r.h->cfg, r.n, 0) > kRanmarWaveMax)
            return fail(PRNGD_ERR_UNSUPPORTED,
                        "request %u: RANMAR plans take requests of at most %llu planned pairs", i,
                        (unsigned long long)kRanmarWaveMax);
        Segment seg{};
        uint64_t ntiles = 0;
        prngd_status_t st = make_segment(r.h, r.n, r.out, kRanmarSegPairs[0], 0, 0, &seg, &ntiles);
        if (st != PRNGD_OK)
            return st;
        seg.seed = reinterpret_cast<uint64_t>(r.h->rm);
        segs.push_back(seg);
        p->handles.push_back(r.h);
    }
    if (segs.empty())
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "a plan needs at least one request with n > 0");
    prngd_status_t st = ws_init(&p->ws, p->device);
    if (st != PRNGD_OK)
        return st;
    for (prngd_handle_t h : p->handles)
        if (h->last_event)
            HIP_TRY(hipEventSynchronize(h->last_event));
    void *dp = nullptr;
    HIP_TRY(hipMalloc(&dp, segs.size() * sizeof(Segment)));
    p->dsegs = static_cast<Segment *>(dp);
    HIP_TRY(hipMalloc(&dp, sizeof(uint32_t)));
    p->flip = static_cast<uint32_t *>(dp);
    HIP_TRY(hipMemcpy(p->dsegs, segs.data(), segs.size() * sizeof(Segment),
                      hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(p->flip, 0, sizeof(uint32_t)));
    HIP_TRY(hipDeviceSynchronize());
    p->spec = true;                          // no look-back status words to renew
    p->lb_args = ranmar_args(d, first->cfg);
    p->lb_args.segs = p->dsegs;
    p->lb_args.nseg = uint32_t(segs.size());
    p->lb_args.total_tiles = uint32_t(segs.size());
    p->lb_args.flip = p->flip;
    HIP_TRY(hipGraphCreate(&p->graph, 0));
    hipKernelNodeParams kp{};
    void *params[] = {&p->lb_args};
    kp.func = const_cast<void *>(ranmar_kernel_for(ranmar_kfam(first->cfg), 0));
    kp.gridDim = dim3(uint32_t((segs.size() + 3) / 4));
    kp.blockDim = dim3(256);
    kp.kernelParams = params;
    hipGraphNode_t fill_node, toggle_node;
    HIP_TRY(hipGraphAddKernelNode(&fill_node, p->graph, nullptr, 0, &kp));
    uint32_t *flip = p->flip;
    void *tparams[] = {&flip};
    hipKernelNodeParams tp{};
    tp.func = const_cast<void *>(toggle_flip_kernel_ptr());
    tp.gridDim = dim3(1);
    tp.blockDim = dim3(1);
    tp.kernelParams = tparams;
    HIP_TRY(hipGraphAddKernelNode(&toggle_node, p->graph, &fill_node, 1, &tp));
    HIP_TRY(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    p->ws.launches = 0;
    for (size_t i = 0; i < p->handles.size(); ++i) {
        prngd_handle_t h = p->handles[i];
        p->base_parity.push_back(h->parity);
        h->plan = p.get();
        h->plan_index = i;
    }
    *out_plan = p.release();
    return PRNGD_OK;
}

prngd_status_t prngd_fill(prngd_handle_t h, uint64_t n, double *out, void *stream)
{
    if (!h)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "NULL handle");
    if (h->plan)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "handle is bound to a live plan");
    if (n == 0)
        return PRNGD_OK;
    std::lock_guard<std::recursive_mutex> lock(g_mutex);
    DeviceInfo *d = nullptr;
    prngd_status_t st = device_info(h->device, &d);
    if (st != PRNGD_OK)
        return st;
    if ((st = check_device_errors(d)) != PRNGD_OK)
        return st;
    if (h->cfg.fam == FAM_RANMAR) {
        hipStream_t s = static_cast<hipStream_t>(stream);
        Workspace *ws = nullptr;
        if ((st = stream_workspace(h->device, s, &ws)) != PRNGD_OK)
            return st;
        if ((st = order_after(h, s)) != PRNGD_OK)
            return st;
        if ((st = ranmar_fill(d, h, n, out, ws, s)) != PRNGD_OK)
            return st;
        HIP_TRY(hipEventRecord(ws->last, s));
        h->parity ^= 1u;
        h->last_event = ws->last;
        h->last_stream = s;
        return PRNGD_OK;
    }
    LaunchArgs args{};
    LaunchPlan lp{};
    if ((st = plan_launch(d, h->cfg, &args, &lp)) != PRNGD_OK)
        return st;
    const bool words = h->cfg.consume == PRNGD_CONSUME_SINGLE;
    if (words && !words_spec_wanted(lp, h->cfg, n)) {
        // a one-segment batch: the segment-sequential one-word kernel
        const prngd_request_t r{h, n, out};
        return fill_batch_impl(&r, 1, stream);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace *ws = nullptr;
    if ((st = stream_workspace(h->device, s, &ws)) != PRNGD_OK)
        return st;
    uint64_t ntiles = 0;
    for (int pass = 0; pass < 2; ++pass) {
        if ((st = make_segment(h, n, out, lp.T, lp.tune.slack_mode, 0, &args.seg0, &ntiles)) !=
            PRNGD_OK)
            return st;
        args.nseg = 1;
        args.total_tiles = uint32_t(ntiles);
        args.ctl = ws->ctl;
        choose_path(&lp, h->cfg, args.seg0.planned, args.seg0.planned, true);
        if (pass == 1 || words || !lp.spec || !philox_family(h->cfg.fam) ||
            !ppl_is_default(h->cfg.fam, h->cfg.w))
            break;
        // a speculative single Philox fill: plan again in its own tile size
        // (the wave-granular form in chunks of one window)
        args = LaunchArgs{};
        const bool wave = lp.wave;
        lp = LaunchPlan{};
        if ((st = plan_launch(d, h->cfg, &args, &lp, wave ? kSingleWavePpl : kSingleSpecPpl)) !=
            PRNGD_OK)
            return st;
    }
    if ((st = order_after(h, s)) != PRNGD_OK)
        return st;
    if (words) {
        if ((st = launch_spec_words(d, lp, ws, args, s)) != PRNGD_OK)
            return st;
    } else if (lp.counted) {
        if ((st = launch_counted(lp, ws, args, s)) != PRNGD_OK)
            return st;
    } else if (lp.spec && lp.wave) {
        if ((st = launch_spec_wave(d, lp, ws, args, s)) != PRNGD_OK)
            return st;
    } else if (lp.spec) {
        if ((st = ws_prepare_spec(ws, ntiles, s)) != PRNGD_OK)
            return st;
        if ((st = launch_spec(d, lp, ws, args, ntiles, s)) != PRNGD_OK)
            return st;
    } else {
        if ((st = ws_prepare(ws, ntiles, s)) != PRNGD_OK)
            return st;
        args.status = ws->status;
        HIP_TRY(launch_fill(lp.kernel, grid_for(d, lp, lp.kernel, ntiles), lp.threads, args, s));
        ws->launches++;
    }
    HIP_TRY(hipEventRecord(ws->last, s));
    h->parity ^= 1u;
    h->last_event = ws->last;
    h->last_stream = s;
    return PRNGD_OK;
}

prngd_status_t prngd_fill_noalloc(prngd_handle_t h, uint64_t n, double *out, void *stream)
{
    if (!h)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "NULL handle");
    if (h->plan)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "handle is bound to a live plan");
    if (n == 0)
        return PRNGD_OK;
    std::lock_guard<std::recursive_mutex> lock(g_mutex);
    auto it = g_devices.find(h->device);
    if (it == g_devices.end())
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "handle's device is not set up");
    DeviceInfo *d = &it->second;
    prngd_status_t st = check_device_errors(d);
    if (st != PRNGD_OK)
        return st;
    if (h->cfg.consume != PRNGD_CONSUME_PAIR)
        return fail(PRNGD_ERR_UNSUPPORTED, "prngd_fill_noalloc takes pair consumption only");
    if (h->cfg.fam == FAM_RANMAR)
        return fail(PRNGD_ERR_UNSUPPORTED, "prngd_fill_noalloc takes no RANMAR handles");
    Control *ctl = noalloc_control(h->device);
    uint64_t *status = noalloc_status(h->device);
    if (!ctl || !status)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "handle's device has no fixed scratch");
    LaunchArgs args{};
    LaunchPlan lp{};
    if ((st = plan_launch(d, h->cfg, &args, &lp, 16, false)) != PRNGD_OK)
        return st;
    uint64_t ntiles = 0;
    if ((st = make_segment(h, n, out, lp.T, lp.tune.slack_mode, 0, &args.seg0, &ntiles)) !=
        PRNGD_OK)
        return st;
    const size_t cap = noalloc_status_words();
    if (ntiles > cap)
        return fail(PRNGD_ERR_INVALID_ARGUMENT,
                    "n = %llu needs %llu tiles of %llu pairs; the fixed scratch holds %llu",
                    (unsigned long long)n, (unsigned long long)ntiles,
                    (unsigned long long)lp.T, (unsigned long long)cap);
    hipStream_t s = static_cast<hipStream_t>(stream);
    args.nseg = 1;
    args.total_tiles = uint32_t(ntiles);
    args.ctl = ctl;
    args.status = status;
    // status words carry a 24-bit epoch: clear them before it wraps
    if (d->noalloc_launches > 0 && d->noalloc_launches % kEpochMask == 0)
        HIP_TRY(launch_zero_words(status, cap, s));
    if ((st = order_after(h, s)) != PRNGD_OK)
        return st;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, lp.kernel, int(lp.threads), 0) !=
            hipSuccess || occ <= 0)
        occ = 1;
    const uint64_t per_cu = lp.tune.blocks_per_cu ? lp.tune.blocks_per_cu : uint64_t(occ);
    const uint64_t grid = std::max<uint64_t>(1, std::min<uint64_t>(per_cu * d->cus, ntiles));
    HIP_TRY(launch_fill(lp.kernel, uint32_t(grid), lp.threads, args, s));
    d->noalloc_launches++;
    HIP_TRY(hipEventRecord(d->noalloc_event, s));
    h->parity ^= 1u;
    h->last_event = d->noalloc_event;
    h->last_stream = s;
    return PRNGD_OK;
}

prngd_status_t prngd_fill_batch(const prngd_request_t *reqs, uint32_t count, void *stream)
{
    std::lock_guard<std::recursive_mutex> lock(g_mutex);
    if (!reqs || count == 0)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "empty request list");
    if (!reqs[0].h)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "request 0 has a NULL handle");
    // one request: the single-fill path (no descriptor upload)
    if (count == 1 && reqs[0].h->cfg.consume == PRNGD_CONSUME_PAIR) {
        if (reqs[0].h->plan)
            return fail(PRNGD_ERR_INVALID_ARGUMENT, "request 0: handle bound to a plan");
        return prngd_fill(reqs[0].h, reqs[0].n, reqs[0].out, stream);
    }
    return fill_batch_impl(reqs, count, stream);
}

static prngd_status_t fill_batch_impl(const prngd_request_t *reqs, uint32_t count, void *stream)
{
    std::lock_guard<std::recursive_mutex> lock(g_mutex);
    const int dev = reqs[0].h->device;
    DeviceInfo *d = nullptr;
    prngd_status_t st = device_info(dev, &d);
    if (st != PRNGD_OK)
        return st;
    if ((st = check_device_errors(d)) != PRNGD_OK)
        return st;
    const Config cfg = reqs[0].h->cfg;
    if (cfg.fam == FAM_RANMAR)
        return ranmar_batch(d, reqs, count, static_cast<hipStream_t>(stream));
    LaunchArgs args{};
    LaunchPlan lp{};
    if ((st = plan_launch(d, cfg, &args, &lp)) != PRNGD_OK)
        return st;
    BatchPlan bp;
    if ((st = build_batch(d, lp, reqs, count, &bp)) != PRNGD_OK)
        return st;
    if (bp.handles.empty())
        return PRNGD_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Workspace *ws = nullptr;
    if ((st = stream_workspace(dev, s, &ws)) != PRNGD_OK)
        return st;
    // order after every handle's previous work on other streams
    std::unordered_set<hipEvent_t> waited;
    for (prngd_handle_t h : bp.handles)
        if (h->last_event && h->last_stream != s && waited.insert(h->last_event).second)
            HIP_TRY(hipStreamWaitEvent(s, h->last_event, 0));
    const size_t nseg = bp.lb.size() + bp.seq.size();
    if ((st = lp.chunk  ? ws_prepare_chunk(ws, nseg, s)
              : lp.spec ? ws_prepare_spec(ws, bp.lb_tiles, s)
                        : ws_prepare(ws, bp.lb_tiles, s)) != PRNGD_OK)
        return st;
    if ((st = ws_grow(ws, &ws->dsegs, &ws->dsegs_cap, nseg, s)) != PRNGD_OK)
        return st;
    if ((st = ws_grow(ws, &ws->tile_seg, &ws->tile_seg_cap, std::max<uint64_t>(bp.lb_tiles, 1), s)) !=
        PRNGD_OK)
        return st;
    // descriptors (look-back ones first): pinned staging ring of two, one
    // async copy, then the tile -> segment map is expanded on the device
    const int slot = ws->hcur;
    ws->hcur ^= 1;
    HIP_TRY(hipEventSynchronize(ws->hsegs_done[slot]));
    if (ws->hsegs_cap[slot] < nseg) {
        if (ws->hsegs[slot])
            ws->retired_host.push_back(ws->hsegs[slot]);
        void *p = nullptr;
        const size_t cap = std::max<size_t>({nseg, size_t(1024), 2 * ws->hsegs_cap[slot]});
        HIP_TRY(hipHostMalloc(&p, cap * sizeof(Segment), hipHostMallocDefault));
        ws->hsegs[slot] = static_cast<Segment *>(p);
        ws->hsegs_cap[slot] = cap;
    }
    std::copy(bp.lb.begin(), bp.lb.end(), ws->hsegs[slot]);
    std::copy(bp.seq.begin(), bp.seq.end(), ws->hsegs[slot] + bp.lb.size());
    HIP_TRY(hipMemcpyAsync(ws->dsegs, ws->hsegs[slot], nseg * sizeof(Segment),
                           hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(ws->hsegs_done[slot], s));
    if (!bp.seq.empty()) {
        LaunchArgs sa = args;
        sa.segs = ws->dsegs + bp.lb.size();
        sa.nseg = uint32_t(bp.seq.size());
        sa.total_tiles = uint32_t(bp.seq.size());
        sa.ctl = ws->seq_ctl;
        HIP_TRY(launch_fill(lp.seq_kernel, grid_for(d, lp, lp.seq_kernel, bp.seq.size()),
                            lp.threads, sa, s));
    }
    if (!bp.lb.empty()) {
        if (!lp.chunk || bp.chunks_per_seg == 0)
            HIP_TRY(launch_expand_tiles(ws->dsegs, uint32_t(bp.lb.size()), ws->tile_seg, s));
        args.segs = ws->dsegs;
        args.tile_seg = ws->tile_seg;
        args.nseg = uint32_t(bp.lb.size());
        args.total_tiles = uint32_t(bp.lb_tiles);
        if (lp.chunk) {
            if ((st = launch_chunk(d, lp, ws, args, bp.chunks_per_seg, s)) != PRNGD_OK)
                return st;
        } else if (lp.spec) {
            if ((st = launch_spec(d, lp, ws, args, bp.lb_tiles, s)) != PRNGD_OK)
                return st;
        } else {
            args.status = ws->status;
            args.ctl = ws->ctl;
            HIP_TRY(launch_fill(lp.kernel, grid_for(d, lp, lp.kernel, bp.lb_tiles), lp.threads,
                                args, s));
            ws->launches++;
        }
    }
    HIP_TRY(hipEventRecord(ws->last, s));
    for (prngd_handle_t h : bp.handles) {
        h->parity ^= 1u;
        h->last_event = ws->last;
        h->last_stream = s;
    }
    return PRNGD_OK;
}

prngd_status_t prngd_plan_create(const prngd_request_t *reqs, uint32_t count,
                                 prngd_plan_t *out_plan)
{
    if (!out_plan)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "out_plan is NULL");
    *out_plan = nullptr;
    std::lock_guard<std::recursive_mutex> lock(g_mutex);
    if (!reqs || count == 0 || !reqs[0].h)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "empty request list");
    const int dev = reqs[0].h->device;
    DeviceInfo *d = nullptr;
    prngd_status_t st = device_info(dev, &d);
    if (st != PRNGD_OK)
        return st;
    const Config cfg = reqs[0].h->cfg;
    if (cfg.fam == FAM_RANMAR)
        return ranmar_plan_create(d, reqs, count, out_plan);
    std::unique_ptr<prngd_plan_s> p(new prngd_plan_s);
    p->device = dev;
    LaunchArgs args{};
    LaunchPlan lp{};
    if ((st = plan_launch(d, cfg, &args, &lp)) != PRNGD_OK)
        return st;
    BatchPlan bp;
    if ((st = build_batch(d, lp, reqs, count, &bp)) != PRNGD_OK)
        return st;
    if (bp.handles.empty())
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "a plan needs at least one request with n > 0");
    p->handles = bp.handles;
    if ((st = ws_init(&p->ws, dev)) != PRNGD_OK)
        return st;
    // wait for the handles' earlier work before the plan's first use
    for (prngd_handle_t h : p->handles)
        if (h->last_event)
            HIP_TRY(hipEventSynchronize(h->last_event));
    const size_t nseg = bp.lb.size() + bp.seq.size();
    if ((st = lp.chunk  ? ws_prepare_chunk(&p->ws, nseg, nullptr)
              : lp.spec ? ws_prepare_spec(&p->ws, bp.lb_tiles, nullptr)
                        : ws_prepare(&p->ws, bp.lb_tiles, nullptr)) != PRNGD_OK) {
        ws_release(&p->ws);
        return st;
    }
    std::vector<Segment> all(bp.lb);
    all.insert(all.end(), bp.seq.begin(), bp.seq.end());
    std::vector<uint32_t> map(std::max<uint64_t>(bp.lb_tiles, 1), 0u);
    for (size_t i = 0; i < bp.lb.size(); ++i)
        std::fill(map.begin() + bp.lb[i].tile_begin,
                  map.begin() + bp.lb[i].tile_begin + bp.lb[i].ntiles, uint32_t(i));
    void *dp = nullptr;
    HIP_TRY(hipMalloc(&dp, nseg * sizeof(Segment)));
    p->dsegs = static_cast<Segment *>(dp);
    HIP_TRY(hipMalloc(&dp, map.size() * sizeof(uint32_t)));
    p->tile_seg = static_cast<uint32_t *>(dp);
    HIP_TRY(hipMalloc(&dp, sizeof(uint32_t)));
    p->flip = static_cast<uint32_t *>(dp);
    HIP_TRY(hipMemcpy(p->dsegs, all.data(), nseg * sizeof(Segment), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(p->tile_seg, map.data(), map.size() * sizeof(uint32_t),
                      hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(p->flip, 0, sizeof(uint32_t)));
    HIP_TRY(hipDeviceSynchronize());
    // graph: [sequential kernel] and [look-back kernel] in parallel, then
    // the replay-parity toggle after both
    HIP_TRY(hipGraphCreate(&p->graph, 0));
    std::vector<hipGraphNode_t> fills;
    p->seq_args = args;
    p->seq_args.flip = p->flip;
    p->lb_args = args;
    p->lb_args.flip = p->flip;
    if (!bp.seq.empty()) {
        p->seq_args.segs = p->dsegs + bp.lb.size();
        p->seq_args.nseg = uint32_t(bp.seq.size());
        p->seq_args.total_tiles = uint32_t(bp.seq.size());
        p->seq_args.ctl = p->ws.seq_ctl;
        hipKernelNodeParams kp{};
        void *params[] = {&p->seq_args};
        kp.func = const_cast<void *>(lp.seq_kernel);
        kp.gridDim = dim3(grid_for(d, lp, lp.seq_kernel, bp.seq.size()));
        kp.blockDim = dim3(lp.threads);
        kp.kernelParams = params;
        hipGraphNode_t node;
        HIP_TRY(hipGraphAddKernelNode(&node, p->graph, nullptr, 0, &kp));
        fills.push_back(node);
    }
    if (!bp.lb.empty() && lp.chunk) {
        // chunk-speculative fill: the records, the chunks, the repair
        p->spec = true;
        p->lb_args.segs = p->dsegs;
        p->lb_args.tile_seg = p->tile_seg;
        p->lb_args.nseg = uint32_t(bp.lb.size());
        p->lb_args.total_tiles = uint32_t(bp.lb_tiles);
        p->lb_args = chunk_args(lp, &p->ws, p->lb_args, bp.chunks_per_seg);
        p->lb_args.toggle = p->flip;           // the repair flips the parity last
        hipKernelNodeParams kp{};
        void *params[] = {&p->lb_args};
        kp.func = const_cast<void *>(chunk_prep_kernel_ptr());
        kp.gridDim = dim3((p->lb_args.nseg + 255) / 256);
        kp.blockDim = dim3(256);
        kp.kernelParams = params;
        hipGraphNode_t pnode, cnode, rnode;
        HIP_TRY(hipGraphAddKernelNode(&pnode, p->graph, nullptr, 0, &kp));
        kp.func = const_cast<void *>(lp.chunk_kernel);
        kp.gridDim = dim3(chunk_grid(bp.lb_tiles));
        HIP_TRY(hipGraphAddKernelNode(&cnode, p->graph, &pnode, 1, &kp));
        kp.func = const_cast<void *>(lp.chunk_repair_kernel);
        kp.gridDim = dim3(chunk_repair_grid(d, p->lb_args.nseg, lp.expected_rejections));
        kp.blockDim = dim3(kChunkRepairThreads);
        HIP_TRY(hipGraphAddKernelNode(&rnode, p->graph, &cnode, 1, &kp));
        fills.push_back(rnode);
    } else if (!bp.lb.empty() && lp.spec) {
        // speculative fill, then its repair
        p->spec = true;
        p->lb_args.segs = p->dsegs;
        p->lb_args.tile_seg = p->tile_seg;
        p->lb_args.nseg = uint32_t(bp.lb.size());
        p->lb_args.total_tiles = uint32_t(bp.lb_tiles);
        p->lb_args.spec = p->ws.spec;
        p->lb_args.rejlist = p->ws.rejlist;
        p->lb_args.hint = p->ws.hint;
        hipKernelNodeParams kp{};
        void *params[] = {&p->lb_args};
        kp.func = const_cast<void *>(lp.spec_kernel);
        kp.gridDim = dim3(uint32_t(bp.lb_tiles));
        kp.blockDim = dim3(lp.threads);
        kp.kernelParams = params;
        hipGraphNode_t node, rnode;
        HIP_TRY(hipGraphAddKernelNode(&node, p->graph, nullptr, 0, &kp));
        kp.func = const_cast<void *>(lp.repair_kernel);
        kp.gridDim = dim3(repair_grid(d, lp, bp.lb_tiles));
        HIP_TRY(hipGraphAddKernelNode(&rnode, p->graph, &node, 1, &kp));
        fills.push_back(rnode);
    } else if (!bp.lb.empty()) {
        p->lb_args.segs = p->dsegs;
        p->lb_args.tile_seg = p->tile_seg;
        p->lb_args.nseg = uint32_t(bp.lb.size());
        p->lb_args.total_tiles = uint32_t(bp.lb_tiles);
        p->lb_args.status = p->ws.status;
        p->lb_args.ctl = p->ws.ctl;
        hipKernelNodeParams kp{};
        void *params[] = {&p->lb_args};
        kp.func = const_cast<void *>(lp.kernel);
        kp.gridDim = dim3(grid_for(d, lp, lp.kernel, bp.lb_tiles));
        kp.blockDim = dim3(lp.threads);
        kp.kernelParams = params;
        hipGraphNode_t node;
        HIP_TRY(hipGraphAddKernelNode(&node, p->graph, nullptr, 0, &kp));
        fills.push_back(node);
    }
    if (!(lp.chunk && !bp.lb.empty())) {
        hipKernelNodeParams kp{};
        uint32_t *flip = p->flip;
        void *params[] = {&flip};
        kp.func = const_cast<void *>(toggle_flip_kernel_ptr());
        kp.gridDim = dim3(1);
        kp.blockDim = dim3(1);
        kp.kernelParams = params;
        hipGraphNode_t node;
        HIP_TRY(hipGraphAddKernelNode(&node, p->graph, fills.data(), fills.size(), &kp));
    }
    HIP_TRY(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    p->ws.launches = 0;
    for (size_t i = 0; i < p->handles.size(); ++i) {
        prngd_handle_t h = p->handles[i];
        p->base_parity.push_back(h->parity);
        h->plan = p.get();
        h->plan_index = i;
    }
    p->lb_args.total_tiles = uint32_t(bp.lb_tiles);
    *out_plan = p.release();
    return PRNGD_OK;
}

prngd_status_t prngd_plan_launch(prngd_plan_t p, void *stream)
{
    if (!p)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "NULL plan");
    std::lock_guard<std::recursive_mutex> lock(g_mutex);
    DeviceInfo *d = nullptr;
    prngd_status_t st = device_info(p->device, &d);
    if (st != PRNGD_OK)
        return st;
    if ((st = check_device_errors(d)) != PRNGD_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool has_lb = p->lb_args.total_tiles > 0 && !p->spec;
    if (has_lb && p->ws.launches > 0 && p->ws.launches % kEpochMask == 0)
        HIP_TRY(launch_zero_words(p->ws.status, p->ws.status_cap, s));
    HIP_TRY(hipGraphLaunch(p->exec, s));
    if (has_lb)
        p->ws.launches++;
    p->launches++;
    HIP_TRY(hipEventRecord(p->ws.last, s));
    for (prngd_handle_t h : p->handles) {
        h->last_event = p->ws.last;
        h->last_stream = s;
    }
    return PRNGD_OK;
}

prngd_status_t prngd_plan_destroy(prngd_plan_t p)
{
    if (!p)
        return PRNGD_OK;
    std::lock_guard<std::recursive_mutex> lock(g_mutex);
    HIP_TRY(hipEventSynchronize(p->ws.last));
    for (size_t i = 0; i < p->handles.size(); ++i) {
        prngd_handle_t h = p->handles[i];
        h->parity = p->base_parity[i] ^ uint32_t(p->launches & 1u);
        h->plan = nullptr;
        h->last_event = nullptr;
        h->last_stream = nullptr;
    }
    if (p->exec)
        (void)hipGraphExecDestroy(p->exec);
    if (p->graph)
        (void)hipGraphDestroy(p->graph);
    (void)hipFree(p->dsegs);
    (void)hipFree(p->tile_seg);
    (void)hipFree(p->flip);
    ws_release(&p->ws);
    delete p;
    return PRNGD_OK;
}

prngd_status_t prngd_set_tuning(prngd_generator_t generator, uint32_t w,
                                const prngd_tuning_t *tuning)
{
    if (generator < PRNGD_PHILOX4X32_10 || generator > PRNGD_ENUMERATE)
        return fail(PRNGD_ERR_UNSUPPORTED, "unknown generator %d", int(generator));
    const uint32_t fam = kernel_family(generator, w);
    std::lock_guard<std::recursive_mutex> lock(g_mutex);
    if (!tuning) {
        g_tuning.erase(std::make_pair(fam, w));
        return PRNGD_OK;
    }
    prngd_tuning_t t = *tuning;
    const prngd_tuning_t def = tuning_for(fam, 0xFFFFFFFFu);
    const uint32_t threads = t.block_threads ? t.block_threads : def.block_threads;
    const uint32_t ppl = t.pairs_per_lane ? t.pairs_per_lane : def.pairs_per_lane;
    if (!fill_kernel_for(fam, threads, ppl, false))
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "no kernel for %u threads x %u pairs per lane",
                    threads, ppl);
    if (t.store_mode > 2 || t.slack_mode > 1 || t.path > 6)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "bad store_mode, slack_mode or path");
    if (t.path >= 2 && !spec_kernel_for(fam, threads, ppl, false, false, true))
        return fail(PRNGD_ERR_INVALID_ARGUMENT,
                    "no speculative fill for this generator and launch shape");
    g_tuning[std::make_pair(fam, w)] = t;
    return PRNGD_OK;
}

prngd_status_t prngd_get_tuning(prngd_generator_t generator, uint32_t w, prngd_tuning_t *tuning)
{
    if (generator < PRNGD_PHILOX4X32_10 || generator > PRNGD_ENUMERATE || !tuning)
        return fail(PRNGD_ERR_INVALID_ARGUMENT, "bad arguments");
    std::lock_guard<std::recursive_mutex> lock(g_mutex);
    *tuning = tuning_for(kernel_family(generator, w), w);
    return PRNGD_OK;
}

}  // extern "C"
