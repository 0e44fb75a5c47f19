// 3D (tetrahedron) instantiations of the operator kernels.
#define SDG_SHAPES(X) \
  X(3, 1, 1) X(3, 1, 2) X(3, 1, 3) \
  X(3, 2, 1) X(3, 2, 2) X(3, 2, 3) \
  X(3, 3, 1) X(3, 4, 1)
#define SDG_DISPATCH_NAME dispatch_3d
#include "op_kernels.inc"
