// 2D (triangle) instantiations of the operator kernels.
#define SDG_SHAPES(X) \
  X(2, 1, 1) X(2, 1, 2) X(2, 1, 3) X(2, 1, 4) \
  X(2, 2, 1) X(2, 2, 2) X(2, 2, 3) X(2, 2, 4) \
  X(2, 3, 1) X(2, 3, 2) X(2, 3, 3) X(2, 3, 4) \
  X(2, 4, 1) X(2, 4, 2) X(2, 4, 3) X(2, 4, 4)
#define SDG_DISPATCH_NAME dispatch_2d
#include "op_kernels.inc"
