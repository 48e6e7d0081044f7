// The tied order-2 cluster-box adjoint scatter in the frame of Table 1's
// directions (2,1), (1,2), (1,-2), (2,-1): the kernels of adjoint.hip,
// instantiated in a translation unit of their own so that the two compile in
// parallel.
#define BSF_ADJOINT_FRAME1_UNIT 1
#include "adjoint.hip"
