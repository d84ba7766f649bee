// prngd_k_triple.hip -- three words per output (the paper's Conclusion):
// the ordered look-back and segment-sequential kernels and the counted
// single fill, 256 threads and 16 triples per thread, for the Philox
// families and the test generator.
#include "prngd_device.hpp"

namespace prngd {

// The triple kernel for a family (look-back, or segment-sequential with
// seq), or null.
const void *triple_kernel_for(uint32_t fam, bool seq)
{
    switch (fam_base(fam)) {
    case FAM_PHILOX32:
        return seq ? reinterpret_cast<const void *>(&seq_triple_kernel<4, 4, FAM_PHILOX32>)
                   : reinterpret_cast<const void *>(&fill_triple_kernel<4, 4, FAM_PHILOX32>);
    case FAM_PHILOX:
        return seq ? reinterpret_cast<const void *>(&seq_triple_kernel<4, 4, FAM_PHILOX>)
                   : reinterpret_cast<const void *>(&fill_triple_kernel<4, 4, FAM_PHILOX>);
    case FAM_ENUM:
        return seq ? reinterpret_cast<const void *>(&seq_triple_kernel<4, 4, FAM_ENUM>)
                   : reinterpret_cast<const void *>(&fill_triple_kernel<4, 4, FAM_ENUM>);
    default:
        return nullptr;
    }
}

// The counted fill's counting or producing kernel of triples for a family,
// or null.
const void *counted_triple_kernel_for(uint32_t fam, bool produce)
{
    switch (fam_base(fam)) {
    case FAM_PHILOX32:
        return produce ? reinterpret_cast<const void *>(&counted_triple_kernel<4, 4, FAM_PHILOX32, true>)
                       : reinterpret_cast<const void *>(&counted_triple_kernel<4, 4, FAM_PHILOX32, false>);
    case FAM_PHILOX:
        return produce ? reinterpret_cast<const void *>(&counted_triple_kernel<4, 4, FAM_PHILOX, true>)
                       : reinterpret_cast<const void *>(&counted_triple_kernel<4, 4, FAM_PHILOX, false>);
    case FAM_ENUM:
        return produce ? reinterpret_cast<const void *>(&counted_triple_kernel<4, 4, FAM_ENUM, true>)
                       : reinterpret_cast<const void *>(&counted_triple_kernel<4, 4, FAM_ENUM, false>);
    default:
        return nullptr;
    }
}

}  // namespace prngd
