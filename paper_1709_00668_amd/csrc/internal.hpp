// Library-internal calls on a resident tensor (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "../../include/sambaten.h"

namespace sbt {
// bytes of one element of the dense store (0 for a COO tensor)
size_t store_elem_bytes(const sbt_tensor* t);
// whether the tensor is a third-order COO tensor
bool is_coo(const sbt_tensor* t);
// device bytes an update of the tensor works in: everything the tensor holds
// besides its store, model and importance (summaries, their factors, the
// sampling and ALS buffers, grown COO buffers)
size_t update_workspace_bytes(const sbt_tensor* t);
// the updates a server runs: like sbt_update_batch_*, but allowed while the
// tensor's requests are held by the server
sbt_status server_update_dense(sbt_tensor* t, const void* Y_dev, int64_t K_new, hipStream_t st);
sbt_status server_update_coo(sbt_tensor* t, const int32_t* i_dev, const int32_t* j_dev,
                             const int32_t* k_dev, const float* v_dev, int64_t nnz,
                             int64_t K_new, hipStream_t st);
// requests a server holds of the tensor (+1 at submission, -1 when done)
void server_lease(sbt_tensor* t, int delta);
}  // namespace sbt
