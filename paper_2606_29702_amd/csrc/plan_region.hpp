// Library-internal plan construction in a caller-given device region, used by
// the no-allocation entry point (noalloc.hip).  Not part of the public ABI.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "pinn_jet.h"

namespace pj_host {

// Sets the calling thread's pinn_last_error() message.
void set_error(const char *msg);

// Device bytes of the workspace of a plan for this network, PDE, point count
// and operand type with every layer stored (no save cap).  Validates like
// pinn_plan_create; touches no device.
pinn_status plan_region_bytes(const pinn_net *net, const pinn_pde *pde, int64_t max_points, int32_t prec,
                              size_t *bytes);

// A plan (no save cap, no flags) whose workspace is carved from the device
// region [region, region + region_bytes): nothing is allocated, and
// pinn_plan_destroy frees no device memory.  PINN_ERR_CAP when it does not fit.
pinn_status plan_create_in_region(const pinn_net *net, const pinn_pde *pde, int64_t max_points, int32_t prec,
                                  void *region, size_t region_bytes, pinn_plan *out);

}  // namespace pj_host
