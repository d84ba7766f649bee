// prngd_internal.hpp -- types shared by the host runtime and the fill
// kernels of libprngd (library-internal, not part of the C ABI).
#pragma once

#include <cstdint>

namespace prngd {

// Base-generator families the kernels are specialised for.
enum Family : uint32_t {
    FAM_PHILOX = 0,   // pair p = words 2p, 2p+1 of one Philox4x32-10 stream
    FAM_MRG = 1,      // pair p = MRG32k3a outputs 2p, 2p+1
    FAM_MIXED = 2,    // pair p = (Philox word p, MRG32k3a output p)
    FAM_ENUM = 3,     // pair p = ((p >> w) mod 2^w, p mod 2^w)
    FAM_PHILOX32 = 4, // FAM_PHILOX at w = 32 (x in [0, 2^32 - 1], no shift)
    FAM_RANMAR = 5    // pair p = RANMAR words 2p, 2p+1 (24 bits), from a window in memory
};

// Flag on a kernel's family: the output map's constants come from the
// launch (Eq. (4), or 1 - z).  Kernels without it compute the default
// Eq. (5) map with the constant S alone.
constexpr uint32_t FAM_ANY_MAP = 0x10u;
constexpr uint32_t kFamBaseMask = 0xFu;

constexpr uint32_t fam_base(uint32_t fam)
{
    return fam & kFamBaseMask;
}

constexpr int kMrgBlockThreads = 256;    // MRG kernels: 4 waves of 64 lanes
constexpr int kMaxBlockThreads = 1024;
constexpr int kMrgDigits = 8;            // window index = 8 base-256 digits
constexpr int kMrgMatWords = 18;         // one 3x3 matrix per component

// Tile status words of the decoupled look-back: [epoch:24 | flag:2 | value:38].
constexpr uint32_t kFlagAggregate = 1;   // value = accepted pairs of the tile
constexpr uint32_t kFlagPrefix = 2;      // value = inclusive prefix in segment
constexpr int kValueBits = 38;
constexpr uint64_t kValueMask = (uint64_t(1) << kValueBits) - 1;
constexpr uint32_t kEpochMask = 0xFFFFFFu;
constexpr uint64_t kMaxOutputs = kValueMask;   // per segment (one fill)

// One fill of one handle inside a launch.  80 bytes; an array of these is
// device-resident for batched launches.
struct Segment {
    uint64_t seed;        // Philox key (seed lo, seed hi); RANMAR: device address of
                          // the handle's two state slots (RanmarState)
    uint64_t n;           // outputs wanted
    uint64_t planned;     // pairs the tiles were planned for (host bookkeeping)
    double *out;          // device output, 8-byte aligned
    uint64_t *counter;    // device position slot: two pair counters
    uint32_t stream_id;   // Philox counter word 3; MRG substream
    uint32_t parity;      // read counter[parity ^ flip], write the other
    uint32_t tile_begin;  // first launch-local tile index of the segment
    uint32_t ntiles;      // tiles of the segment; the last one also takes
                          // every window past its own until n outputs
    uint32_t mrg[6];      // MRG32k3a state at position 0 of the substream
};
static_assert(sizeof(Segment) == 80, "Segment layout");

// Per-workspace launch control of the look-back kernel, device memory,
// zero except epoch = 1.  Tickets grow monotonically across launches: a
// launch of N tiles on G workgroups consumes exactly N + G tickets (every
// workgroup ends with one failing draw), and the workgroup that draws the
// last of them moves `base` and `epoch` on for the next launch.  The
// ticket counter has a cache line to itself: every tile draws from it.
struct Control {
    uint64_t ticket;      // next ticket
    uint64_t pad0[15];
    uint64_t base;        // first ticket of the current launch
    uint32_t epoch;       // epoch of the current launch (1 .. 2^24 - 1)
    uint32_t abort;       // set when a look-back stalls: drain the launch
    uint64_t pad1[14];
};
static_assert(sizeof(Control) == 256, "Control layout");

// Per-workspace bookkeeping of the speculative fill, device memory, zero
// between launches: `count` entries of the rejection list were appended by
// the fill kernel; the repair kernel's workgroups count themselves out in
// `done`, and the last one clears the list for the next launch.
struct SpecControl {
    uint32_t count;
    uint32_t pad0[31];
    uint32_t done;
    uint32_t pad1[31];
};
static_assert(sizeof(SpecControl) == 256, "SpecControl layout");

// Rejection-list entry: (launch-local tile + 1) << 32 | rejected pairs of
// that tile's window; 0 is an empty slot.
constexpr uint32_t kHintEntries = 256;    // entries a tile reads for its hint

// Pairs per chunk of the wave-granular forms: one wave of 64 lanes, two
// pairs per lane.  The batch form's chunks hold 1, 2 or 4 such windows.
constexpr uint32_t kChunkPairs = 128;

// Per-segment record of the chunk-speculative batch fill, written by its
// prologue kernel at every launch (the start position changes from launch
// to launch), read by a wave of the chunk kernel in one scalar batch: one
// 64-byte line (a wave's start latency counts: a larger record, say with
// the Philox round keys, measured slower than the scalar adds it saves).
struct ChunkSeg {
    uint64_t seed;
    double *out;
    uint64_t w0;              // first chunk of the segment (absolute)
    uint64_t n;
    uint64_t *next_counter;   // the position slot half this launch writes
    uint32_t stream_id;
    uint32_t lo0;             // pairs of chunk w0 before the start position
    uint32_t tile_begin;      // first launch-local chunk of the segment
    uint32_t ntiles;          // its chunks; the last one continues until n
    uint32_t k_full;          // chunks below k_full hold P outputs below n - 1
    uint32_t k_end;           // chunks from k_end on hold no output
};
static_assert(sizeof(ChunkSeg) == 64, "ChunkSeg layout");

struct LaunchArgs {
    const Segment *segs;      // nseg descriptors, or null for seg0
    const uint32_t *tile_seg; // launch-local tile -> segment index (segs only)
    Segment seg0;             // the descriptor when segs is null
    uint32_t nseg;
    uint32_t total_tiles;
    uint64_t *status;         // total_tiles status words
    Control *ctl;
    uint32_t *error;          // host-mapped error word
    const uint32_t *flip;     // replay parity of a resident plan, or null
    uint32_t store_mode;      // 0 default, 1 8-byte stores, 2 nontemporal
    uint32_t w;
    uint32_t a0, a;           // x1 range [a0, a]
    uint32_t b0;              // x2 lower bound
    double S;                 // RN((1 - 2^-2w) / D), or RN(1 / D4) for Eq. (4)
    double nadd;              // added to N: 0, or 2^w - (b - b0) for Eq. (4)
    double osign, ooff;       // output = osign * z + ooff: (1, 0), or (-1, 1) for 1 - z
    SpecControl *spec;        // speculative fill: list control,
    uint64_t *rejlist;        //   rejection list (total_tiles slots; list_cap
                              //   slots in the one-word form's candidate list),
    uint32_t *hint;           //   per tile: earlier rejections it assumed
    uint32_t list_cap;        // slots of rejlist
    uint64_t *hint64;         // wave-granular form: per chunk, written only
                              //   when nonzero, (epoch << 24) | rejections
    uint64_t epoch;           // launch number of the workspace (from 1)
    const uint32_t *mrg_thread;  // [256][18]: A^(r * tid * PPL)
    const uint32_t *mrg_window;  // [8][256][18]: A^(r * T * d * 256^i)
    // chunk-speculative batch fill
    ChunkSeg *chunk_segs;     // nseg records
    uint32_t *first_dirty;    // per segment: ~(first chunk with a rejection), 0 = none
    uint32_t *dirty_list;     // segments with a rejection, spec->count of them
    uint32_t chunks_per_seg;  // every segment's chunk count when they are all equal, else 0
    uint32_t cps_magic;       // c / chunks_per_seg as (t + ((c - t) >> 1)) >> cps_shift,
    uint32_t cps_shift;       // t = mulhi(c, cps_magic) (chunks_per_seg >= 2)
    uint32_t chunk_shift;     // log2 of the pairs per chunk
    uint32_t *toggle;         // plan replay parity the chunk repair flips last, or null
    // counted single fill: accepted pairs per chunk, each chunk's offset in
    // its block of kScanBlock chunks, and the blocks' exclusive offsets
    uint32_t *chunk_counts;
    uint32_t *chunk_offs;
    uint64_t *block_offs;
    // RANMAR fills: the jump table (row g, kRanmarRow words: the
    // coefficients of x^(2 g P) mod (x^97 + x^64 - 1) over the integers mod
    // 2^24, then (2 g P * 7654321) mod 16777213) and the pairs P of a segment
    const uint32_t *ranmar_jump;
    uint32_t ranmar_seg_pairs;
    uint32_t spin_limit;      // polls of a look-back wait before a stall (0: kSpinLimit)
};

// Polls of a look-back wait before it reports a stall.
constexpr uint32_t kSpinLimit = 1u << 20;

// RANMAR (Marsaglia, Zaman, Tsang 1990) in integer units of 2^-24: lagged
// values L[n] = (L[n-97] - L[n-33]) mod 2^24, an arithmetic part C[n] =
// (C[n-1] - 7654321) mod 16777213, word j = (L[j+1] - C[j+1]) mod 2^24.
// A handle's state at word position W = 2 * pair counter: L[W-96 .. W] and
// C[W], in one of two slots (read slot parity, write the other, as the
// pair counters).
constexpr uint32_t kRanmarMask = 0xFFFFFFu;
constexpr uint32_t kRanmarCD = 7654321u;
constexpr uint32_t kRanmarCM = 16777213u;
constexpr uint32_t kRanmarC0 = 362436u;
constexpr uint32_t kRanmarRow = 128;       // words of a state slot and of a jump-table row
struct RanmarState {
    uint32_t slot[2][kRanmarRow];          // [0..96] L[W-96 .. W], [97] C[W]
};
// One state to set: both slots of dst, and both pair counters of slot when
// it is not null.
struct RanmarInit {
    RanmarState *dst;
    uint64_t *slot;
    uint64_t counter;
    uint32_t words[kRanmarRow];
};

// Chunks per block of the counted fill's two-level scan (one workgroup of
// 1024 threads, 4 chunks each), and the most blocks its top level takes.
constexpr uint32_t kScanBlock = 4096;
constexpr uint32_t kScanBlocksMax = 1024;

constexpr uint32_t kMaxTiles = 0xFFFFFFF0u;

// Kernel lookup of each kernel translation unit, for a family with the
// map flag MAPF (0 or FAM_ANY_MAP); null for shapes that are not
// instantiated.  The runtime goes through the routers of prngd_k_misc.hip,
// which pick MAPF from the family.
template <uint32_t MAPF>
const void *philox_fill_kernel_for(uint32_t fam, uint32_t threads, uint32_t ppl, bool seq);
template <uint32_t MAPF>
const void *philox_spec_kernel_for(uint32_t fam, uint32_t threads, uint32_t ppl, bool repair,
                                   bool single, bool hold);
template <uint32_t MAPF>
const void *philox_wave_kernel_for(uint32_t fam, bool repair, uint32_t windows);
template <uint32_t MAPF>
const void *mrg_fill_kernel_for(uint32_t fam, uint32_t ppl, bool seq);
template <uint32_t MAPF>
const void *mrg_spec_kernel_for(uint32_t fam, uint32_t ppl, bool repair, bool single);
template <uint32_t MAPF>
const void *single_kernel_for(uint32_t fam);
template <uint32_t MAPF>
const void *spec_words_kernel_for(uint32_t fam, bool repair);
template <uint32_t MAPF>
const void *philox_chunk_kernel_for(uint32_t fam, bool repair, uint32_t windows);
template <uint32_t MAPF>
const void *philox_counted_kernel_for(uint32_t fam, bool produce);
// RANMAR: mode 0 one wave per request (batches, short fills), 1 count the
// accepted pairs of each segment, 2 produce each segment at its offset
template <uint32_t MAPF>
const void *ranmar_kernel_for(uint32_t mode);

// RANMAR on the host: the sequence (ij, kl) of a stream, the state (window
// and C, kRanmarRow words) at word position word_hi 2^64 + word_lo, and
// rows [first, first + count) of the jump table for segments of seg_pairs
// pairs (kRanmarRow words each).
void ranmar_sequence_of(uint64_t seed, uint32_t stream, uint32_t *ij, uint32_t *kl);
void ranmar_window_at(uint64_t seed, uint32_t stream, uint64_t word_lo, uint64_t word_hi,
                      uint32_t out[kRanmarRow]);
void ranmar_jump_rows(uint32_t seg_pairs, uint32_t first, uint32_t count, uint32_t *rows);

// Device error codes (bit flags in the error word).
constexpr uint32_t kErrLookbackStall = 1;
constexpr uint32_t kErrSpecList = 2;       // rejection list out of its bounds
constexpr uint32_t kErrRanmarRunaway = 4;  // a RANMAR wave passed its bound on windows

}  // namespace prngd
