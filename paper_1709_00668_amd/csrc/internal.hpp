// Library-internal queries on a resident tensor (not part of the C ABI).
#pragma once

#include <stddef.h>

#include "../../include/sambaten.h"

namespace sbt {
// bytes of one element of the dense store (0 for a COO tensor)
size_t store_elem_bytes(const sbt_tensor* t);
}  // namespace sbt
