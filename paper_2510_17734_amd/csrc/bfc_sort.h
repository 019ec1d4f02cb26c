// Device prefix sum and stable radix sort used when an observed set is laid out.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bfc {

hipError_t exclusive_scan_i32(int32_t* data, int64_t len, int32_t* scratch, hipStream_t st);
int64_t scan_scratch_elems(int64_t len);
int64_t radix_scratch_bytes(int64_t n);
hipError_t radix_sort_pairs(uint32_t* keys, int32_t* vals, int64_t n, int bits, void* scratch,
                            hipStream_t st);

}  // namespace bfc
