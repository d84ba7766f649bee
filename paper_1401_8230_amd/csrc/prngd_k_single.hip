// prngd_k_single.hip -- Algorithm 1's one-word consumption: the per-request
// kernel, and the one-long-request kernel spread over workgroups with its
// repair pass.  Built twice: with PRNGD_MAPF = 0 (the Eq. (5) kernels) and
// PRNGD_MAPF = FAM_ANY_MAP.
#include "prngd_device.hpp"

namespace prngd {

// The single-word-consumption kernel for a single-generator stream (256
// threads), or null.
template <>
const void *single_kernel_for<PRNGD_MAPF>(uint32_t fam)
{
    constexpr uint32_t P = FAM_PHILOX | PRNGD_MAPF, P32 = FAM_PHILOX32 | PRNGD_MAPF,
                       EN = FAM_ENUM | PRNGD_MAPF, M = FAM_MRG | PRNGD_MAPF;
    switch (fam_base(fam)) {
    case FAM_PHILOX: return reinterpret_cast<const void *>(&seq_single_kernel<4, P>);
    case FAM_PHILOX32: return reinterpret_cast<const void *>(&seq_single_kernel<4, P32>);
    case FAM_ENUM: return reinterpret_cast<const void *>(&seq_single_kernel<4, EN>);
    case FAM_MRG: return reinterpret_cast<const void *>(&seq_single_kernel<4, M>);
    default: return nullptr;
    }
}

// The one-word-consumption speculative fill of one segment across
// workgroups (256 threads), or its repair pass; null for other families.
template <>
const void *spec_words_kernel_for<PRNGD_MAPF>(uint32_t fam, bool repair)
{
    constexpr uint32_t P = FAM_PHILOX | PRNGD_MAPF, P32 = FAM_PHILOX32 | PRNGD_MAPF,
                       EN = FAM_ENUM | PRNGD_MAPF, M = FAM_MRG | PRNGD_MAPF;
    switch (fam_base(fam)) {
    case FAM_PHILOX:
        return repair ? reinterpret_cast<const void *>(&spec_words_repair_kernel<4, P>)
                      : reinterpret_cast<const void *>(&spec_words_kernel<4, P>);
    case FAM_PHILOX32:
        return repair ? reinterpret_cast<const void *>(&spec_words_repair_kernel<4, P32>)
                      : reinterpret_cast<const void *>(&spec_words_kernel<4, P32>);
    case FAM_ENUM:
        return repair ? reinterpret_cast<const void *>(&spec_words_repair_kernel<4, EN>)
                      : reinterpret_cast<const void *>(&spec_words_kernel<4, EN>);
    case FAM_MRG:
        return repair ? reinterpret_cast<const void *>(&spec_words_repair_kernel<4, M>)
                      : reinterpret_cast<const void *>(&spec_words_kernel<4, M>);
    default: return nullptr;
    }
}

}  // namespace prngd
