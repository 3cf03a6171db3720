// Device-wide exclusive prefix sum (host interface).
#pragma once

#include "common.h"

namespace sbx {

// Scratch elements exclusive_scan_u32 needs for n items.
size_t scan_tmp_elems(size_t n);

// In-place exclusive scan of d[0..n); tmp holds scan_tmp_elems(n) uint32.
sbx_status exclusive_scan_u32(uint32_t* d, size_t n, uint32_t* tmp, hipStream_t s);

}  // namespace sbx
