// HSS / URV factor storage of a plan.
#pragma once

#include "plan.h"

namespace nd {

struct HSSFactors {
  virtual ~HSSFactors() = default;
};

int tree_depth(int nx, int ny, int leaf);
void host_binning(const double* points, int64_t M, int nx, int ny, int leaf,
                  int64_t* perm2d, int64_t* leaf_rows, int64_t* colperm);

}  // namespace nd
