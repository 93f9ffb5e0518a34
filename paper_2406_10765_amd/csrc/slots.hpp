// Resources a request-loop slot keeps for its whole life and lends to the handle of each request
// it runs: creating and destroying a rocBLAS handle, a stream and events per request costs host
// time and device allocations while other requests' kernels are in flight.
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include "../../include/pw.h"

namespace pw {

struct SlotResources {
  rocblas_handle blas = nullptr;  // bound to the slot's stream
  hipStream_t aux = nullptr;      // second stream of the H application's local part
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

// Create the resources for a slot whose requests run on `stream`; PW_EDEVICE on failure (nothing
// is left allocated).
pw_status slot_resources_create(hipStream_t stream, SlotResources* r);
void slot_resources_destroy(SlotResources* r);

// pw_setup with the slot's resources lent to the handle (res == nullptr: the handle creates its
// own, as pw_setup does).  The stream must be the one res->blas is bound to.  pw_destroy leaves
// lent resources to the slot.
pw_status setup_handle(const pw_cell_desc* desc, void* arena_dev, size_t arena_bytes, void* hip_stream,
                       const SlotResources* res, pw_handle** out);

}  // namespace pw
