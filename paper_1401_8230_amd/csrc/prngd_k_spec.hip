// prngd_k_spec.hip -- the speculative Philox-family fill kernels (one-shot
// grids with rejection-list hints), their repair pass, and the
// wave-granular single-fill form.  Built twice: with PRNGD_MAPF = 0 (the
// Eq. (5) kernels) and PRNGD_MAPF = FAM_ANY_MAP.
#include "prngd_device.hpp"

namespace prngd {
namespace {

template <int NW, int PPL, uint32_t FAM>
const void *spec_pair(bool repair, bool single, bool hold)
{
    if (repair)
        return reinterpret_cast<const void *>(&spec_repair_kernel<PhiloxRedo<NW, PPL, FAM>>);
    if (hold)
        return single ? reinterpret_cast<const void *>(&spec_hold_kernel<NW, PPL, FAM, true>)
                      : reinterpret_cast<const void *>(&spec_hold_kernel<NW, PPL, FAM, false>);
    return single ? reinterpret_cast<const void *>(&spec_philox_kernel<NW, PPL, FAM, true>)
                  : reinterpret_cast<const void *>(&spec_philox_kernel<NW, PPL, FAM, false>);
}

template <int NW, int PPL>
const void *spec_family(uint32_t fam, bool repair, bool single, bool hold)
{
    switch (fam_base(fam)) {
    case FAM_ENUM: return spec_pair<NW, PPL, FAM_ENUM | PRNGD_MAPF>(repair, single, hold);
    case FAM_PHILOX32: return spec_pair<NW, PPL, FAM_PHILOX32 | PRNGD_MAPF>(repair, single, hold);
    default: return spec_pair<NW, PPL, FAM_PHILOX | PRNGD_MAPF>(repair, single, hold);
    }
}

}  // namespace

template <>
const void *philox_spec_kernel_for<PRNGD_MAPF>(uint32_t fam, uint32_t threads, uint32_t ppl,
                                               bool repair, bool single, bool hold)
{
    if (threads == 256) {
        switch (ppl) {
        case 2: return spec_family<4, 2>(fam, repair, single, hold);
        case 4: return spec_family<4, 4>(fam, repair, single, hold);
        case 8: return spec_family<4, 8>(fam, repair, single, hold);
        case 16: return spec_family<4, 16>(fam, repair, single, hold);
        case 32: return spec_family<4, 32>(fam, repair, single, hold);
        default: return nullptr;
        }
    }
    if (threads == 512) {
        switch (ppl) {
        case 8: return spec_family<8, 8>(fam, repair, single, hold);
        case 16: return spec_family<8, 16>(fam, repair, single, hold);
        default: return nullptr;
        }
    }
    if (threads == 1024) {
        switch (ppl) {
        case 8: return spec_family<16, 8>(fam, repair, single, hold);
        case 16: return spec_family<16, 16>(fam, repair, single, hold);
        default: return nullptr;
        }
    }
    return nullptr;
}

// The wave-granular speculative fill of a single segment in chunks of
// `windows` 128-pair windows (1, 2 or 4), or its repair, for a
// Philox-family generator; null for other families and chunk sizes.
template <uint32_t F>
const void *wave_for(uint32_t windows, bool repair)
{
    switch (windows) {
    case 1:
        return repair ? reinterpret_cast<const void *>(&spec_wave_repair_kernel<F, 1>)
                      : reinterpret_cast<const void *>(&spec_wave_kernel<F, 1>);
    case 2:
        return repair ? reinterpret_cast<const void *>(&spec_wave_repair_kernel<F, 2>)
                      : reinterpret_cast<const void *>(&spec_wave_kernel<F, 2>);
    case 4:
        return repair ? reinterpret_cast<const void *>(&spec_wave_repair_kernel<F, 4>)
                      : reinterpret_cast<const void *>(&spec_wave_kernel<F, 4>);
    default:
        return nullptr;
    }
}

template <>
const void *philox_wave_kernel_for<PRNGD_MAPF>(uint32_t fam, bool repair, uint32_t windows)
{
    switch (fam_base(fam)) {
    case FAM_PHILOX32:
        return wave_for<FAM_PHILOX32 | PRNGD_MAPF>(windows, repair);
    case FAM_PHILOX:
        return wave_for<FAM_PHILOX | PRNGD_MAPF>(windows, repair);
    case FAM_ENUM:
        return wave_for<FAM_ENUM | PRNGD_MAPF>(windows, repair);
    default:
        return nullptr;
    }
}

// The chunk-speculative batch fill of a Philox-family generator in chunks
// of `windows` 128-pair windows (1, 2 or 4), or its repair; null for other
// families and chunk sizes.
template <uint32_t F>
const void *chunk_for(uint32_t windows, bool repair)
{
    switch (windows) {
    case 1:
        return repair ? reinterpret_cast<const void *>(&chunk_repair_kernel<F, 1>)
                      : reinterpret_cast<const void *>(&chunk_batch_kernel<F, 1>);
    case 2:
        return repair ? reinterpret_cast<const void *>(&chunk_repair_kernel<F, 2>)
                      : reinterpret_cast<const void *>(&chunk_batch_kernel<F, 2>);
    case 4:
        return repair ? reinterpret_cast<const void *>(&chunk_repair_kernel<F, 4>)
                      : reinterpret_cast<const void *>(&chunk_batch_kernel<F, 4>);
    default:
        return nullptr;
    }
}

template <>
const void *philox_chunk_kernel_for<PRNGD_MAPF>(uint32_t fam, bool repair, uint32_t windows)
{
    switch (fam_base(fam)) {
    case FAM_PHILOX32:
        return chunk_for<FAM_PHILOX32 | PRNGD_MAPF>(windows, repair);
    case FAM_PHILOX:
        return chunk_for<FAM_PHILOX | PRNGD_MAPF>(windows, repair);
    case FAM_ENUM:
        return chunk_for<FAM_ENUM | PRNGD_MAPF>(windows, repair);
    default:
        return nullptr;
    }
}

// The counted single fill's counting pass or producing pass for a
// Philox-family generator; null for other families.
template <>
const void *philox_counted_kernel_for<PRNGD_MAPF>(uint32_t fam, bool produce)
{
    constexpr uint32_t P32 = FAM_PHILOX32 | PRNGD_MAPF, P = FAM_PHILOX | PRNGD_MAPF,
                       EN = FAM_ENUM | PRNGD_MAPF;
    switch (fam_base(fam)) {
    case FAM_PHILOX32:
        return produce ? reinterpret_cast<const void *>(&counted_produce_kernel<P32>)
                       : reinterpret_cast<const void *>(&counted_count_kernel<P32>);
    case FAM_PHILOX:
        return produce ? reinterpret_cast<const void *>(&counted_produce_kernel<P>)
                       : reinterpret_cast<const void *>(&counted_count_kernel<P>);
    case FAM_ENUM:
        return produce ? reinterpret_cast<const void *>(&counted_produce_kernel<EN>)
                       : reinterpret_cast<const void *>(&counted_count_kernel<EN>);
    default:
        return nullptr;
    }
}

}  // namespace prngd
