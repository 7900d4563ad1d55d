// pc_kernels_t128.hip -- the counting kernels for 128-point tiles (2 i-points
// per lane), namespace pc::t128; the launch picks a tile size at run time.
#define PC_R 2
#include "pc_kernels.hip"
