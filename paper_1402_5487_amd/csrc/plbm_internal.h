// Internal declarations shared by the host and device translation units of
// libplbm (not part of the public ABI).
#pragma once
#include "plbm.h"

namespace plbm {
int nq(const plbm_desc *d);
int validate(const plbm_desc *d);
} // namespace plbm
