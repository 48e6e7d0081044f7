// The tied order-2 cluster-box gather in the frame of Table 1's directions
// (2,1), (1,2), (1,-2), (2,-1): the kernels of gather.hip, instantiated in a
// translation unit of their own so that the two compile in parallel.
#define BSF_GATHER_FRAME1_UNIT 1
#include "gather.hip"
