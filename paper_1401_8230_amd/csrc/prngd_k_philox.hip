// prngd_k_philox.hip -- the ordered Philox-family fill kernels (look-back
// and segment-sequential) for every launch shape.  Built twice: with
// PRNGD_MAPF = 0 (the Eq. (5) kernels) and PRNGD_MAPF = FAM_ANY_MAP.
#include "prngd_device.hpp"

namespace prngd {
namespace {

template <int NW, int PPL, uint32_t FAM>
const void *philox_kernel(bool seq)
{
    return seq ? reinterpret_cast<const void *>(&seq_philox_kernel<NW, PPL, FAM>)
               : reinterpret_cast<const void *>(&fill_philox_kernel<NW, PPL, FAM>);
}

template <int NW, int PPL>
const void *philox_family(uint32_t fam, bool seq)
{
    switch (fam_base(fam)) {
    case FAM_ENUM: return philox_kernel<NW, PPL, FAM_ENUM | PRNGD_MAPF>(seq);
    case FAM_PHILOX32: return philox_kernel<NW, PPL, FAM_PHILOX32 | PRNGD_MAPF>(seq);
    default: return philox_kernel<NW, PPL, FAM_PHILOX | PRNGD_MAPF>(seq);
    }
}

}  // namespace

template <>
const void *philox_fill_kernel_for<PRNGD_MAPF>(uint32_t fam, uint32_t threads, uint32_t ppl,
                                              bool seq)
{
    if (threads == 256) {
        switch (ppl) {
        case 2: return philox_family<4, 2>(fam, seq);
        case 4: return philox_family<4, 4>(fam, seq);
        case 8: return philox_family<4, 8>(fam, seq);
        case 16: return philox_family<4, 16>(fam, seq);
        case 32: return philox_family<4, 32>(fam, seq);
        default: return nullptr;
        }
    }
    if (threads == 512) {
        switch (ppl) {
        case 8: return philox_family<8, 8>(fam, seq);
        case 16: return philox_family<8, 16>(fam, seq);
        default: return nullptr;
        }
    }
    if (threads == 1024) {
        switch (ppl) {
        case 8: return philox_family<16, 8>(fam, seq);
        case 16: return philox_family<16, 16>(fam, seq);
        default: return nullptr;
        }
    }
    return nullptr;
}

}  // namespace prngd
