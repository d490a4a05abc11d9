// Radix sort of (cell key, particle index) pairs with rocPRIM; the key
// extraction and the permutation of the particle arrays are relpic kernels.
#include <rocprim/device/device_radix_sort.hpp>

#include "batch_kernels.h"

namespace relpic {

hipError_t sort_pairs(void *temp, size_t &temp_bytes, const unsigned *keys_in, unsigned *keys_out,
                      const unsigned *idx_in, unsigned *idx_out, long long n, hipStream_t st) {
  return rocprim::radix_sort_pairs(temp, temp_bytes, keys_in, keys_out, idx_in, idx_out, (size_t)n, 0u, 32u, st);
}

// keys below 2^end_bit: only the low end_bit bits are sorted
hipError_t sort_pairs_bits(void *temp, size_t &temp_bytes, const unsigned *keys_in, unsigned *keys_out,
                           const unsigned *idx_in, unsigned *idx_out, long long n, int end_bit, hipStream_t st) {
  return rocprim::radix_sort_pairs(temp, temp_bytes, keys_in, keys_out, idx_in, idx_out, (size_t)n, 0u,
                                   (unsigned)end_bit, st);
}

}  // namespace relpic
