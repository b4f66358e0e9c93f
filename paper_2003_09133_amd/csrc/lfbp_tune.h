// Tuned kernel choices for the H -> H' re-arrangement.
#pragma once

#include "lfbp.h"

namespace lfbp {

// Row class of a shape: floor(log2(ny*nz*esize)), the size class of one
// x-row in bytes, which keys the tuning table.
int row_class(const lfbp_shape& s, int esize);

// The configuration for one problem: the tuning-table entry of its exact
// shape, else of its row class (batched or plain) or of the nearest class
// present, else the built-in defaults.  Every field is set except grid, which may be 0 (= one workgroup
// per unit, or every workgroup slot of the device when persistent).
lfbp_gather_config tuned_config(const lfbp_shape& s, int esize, bool batched);

}  // namespace lfbp
