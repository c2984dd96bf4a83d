// unet.h -- internal interface of the U-Net preconditioner (unet.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fem.h"

namespace fem {

struct UNet;

// z = N(r) on the structured (grid_n + 1)^2 nodal grid: the interior residual,
// scaled to unit RMS, forms an image with a constant second channel `cval`;
// the network output is written back to the interior nodes, boundary nodes and
// nodes with mask[g] != 0 get 0.  Enqueued on `st`; allocates nothing.
int unet_grid_precondition(fem_unet *net, int grid_n, const double *r, double cval, const uint8_t *mask, double *z,
                           hipStream_t st);

}  // namespace fem
