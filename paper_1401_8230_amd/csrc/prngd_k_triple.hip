// prngd_k_triple.hip -- three words per output (the paper's Conclusion):
// the ordered look-back and segment-sequential kernels, 256 threads and 16
// triples per thread, for the Philox families and the test generator.
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

}  // namespace prngd
