// pc_prep_t128.hip -- tile bounds and the prune pass for 128-point tiles,
// namespace pc::t128; the launch picks a tile size at run time.
#define PC_R 2
#include "pc_prep.hip"
