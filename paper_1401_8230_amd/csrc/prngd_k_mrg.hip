// prngd_k_mrg.hip -- the MRG32k3a and mixed Philox/MRG32k3a fill kernels:
// ordered (look-back and segment-sequential), speculative, and the repair
// pass.  Built twice: with PRNGD_MAPF = 0 (the Eq. (5) kernels) and
// PRNGD_MAPF = FAM_ANY_MAP.
#include "prngd_device.hpp"

namespace prngd {
namespace {

template <int PPL>
const void *mrg_family(uint32_t fam, bool seq)
{
    constexpr uint32_t M = FAM_MRG | PRNGD_MAPF, X = FAM_MIXED | PRNGD_MAPF;
    const bool mrg = fam_base(fam) == FAM_MRG;
    if (seq)
        return mrg ? reinterpret_cast<const void *>(&seq_mrg_kernel<PPL, M>)
                   : reinterpret_cast<const void *>(&seq_mrg_kernel<PPL, X>);
    return mrg ? reinterpret_cast<const void *>(&fill_mrg_kernel<PPL, M>)
               : reinterpret_cast<const void *>(&fill_mrg_kernel<PPL, X>);
}

template <int PPL, uint32_t FAM>
const void *spec_mrg_pair(bool repair, bool single)
{
    if (repair)
        return reinterpret_cast<const void *>(&spec_repair_kernel<MrgRedo<PPL, FAM>>);
    return single ? reinterpret_cast<const void *>(&spec_mrg_kernel<PPL, FAM, true>)
                  : reinterpret_cast<const void *>(&spec_mrg_kernel<PPL, FAM, false>);
}

template <int PPL>
const void *spec_mrg_family(uint32_t fam, bool repair, bool single)
{
    return fam_base(fam) == FAM_MRG ? spec_mrg_pair<PPL, FAM_MRG | PRNGD_MAPF>(repair, single)
                                    : spec_mrg_pair<PPL, FAM_MIXED | PRNGD_MAPF>(repair, single);
}

}  // namespace

template <>
const void *mrg_fill_kernel_for<PRNGD_MAPF>(uint32_t fam, uint32_t ppl, bool seq)
{
    switch (ppl) {
    case 4: return mrg_family<4>(fam, seq);
    case 8: return mrg_family<8>(fam, seq);
    case 16: return mrg_family<16>(fam, seq);
    default: return nullptr;
    }
}

template <>
const void *mrg_spec_kernel_for<PRNGD_MAPF>(uint32_t fam, uint32_t ppl, bool repair,
                                            bool single)
{
    switch (ppl) {
    case 4: return spec_mrg_family<4>(fam, repair, single);
    case 8: return spec_mrg_family<8>(fam, repair, single);
    case 16: return spec_mrg_family<16>(fam, repair, single);
    default: return nullptr;
    }
}

}  // namespace prngd
