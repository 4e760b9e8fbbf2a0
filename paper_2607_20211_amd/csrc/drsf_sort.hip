// Device radix sort of 64-bit keys (hipCUB), used when the edge store is
// rebuilt.  Kept in its own file so that only this unit compiles hipCUB.
#include <hipcub/hipcub.hpp>

#include "drsf_kernels.h"

namespace drsf {

size_t sort_u64_tmp_bytes(int64_t count) {
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortKeys(nullptr, bytes, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                            (int)count, 0, 64, (hipStream_t)0);
    return bytes;
}

int launch_sort_u64(const uint64_t *in, uint64_t *out, int64_t count, void *tmp, size_t tmp_bytes,
                    hipStream_t s) {
    size_t bytes = tmp_bytes;
    return hipcub::DeviceRadixSort::SortKeys(tmp, bytes, in, out, (int)count, 0, 64, s) == hipSuccess ? 0 : -1;
}

size_t sort_pairs_u64_tmp_bytes(int64_t count) {
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                             (const uint64_t *)nullptr, (uint64_t *)nullptr, (int)count, 0, 64,
                                             (hipStream_t)0);
    return bytes;
}

int launch_sort_pairs_u64(const uint64_t *kin, uint64_t *kout, const uint64_t *vin, uint64_t *vout,
                          int64_t count, void *tmp, size_t tmp_bytes, hipStream_t s) {
    size_t bytes = tmp_bytes;
    return hipcub::DeviceRadixSort::SortPairs(tmp, bytes, kin, kout, vin, vout, (int)count, 0, 64, s) ==
                   hipSuccess
               ? 0
               : -1;
}

}  // namespace drsf
