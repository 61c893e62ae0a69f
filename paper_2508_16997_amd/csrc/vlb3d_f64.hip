// vlb3d_f64.hip -- the FP64 half of the three-dimensional kernels: vlb3d.hip compiled
// with VLB3_PART 2, which keeps only the double-precision instantiations and the three
// functions of namespace vlb3_f64 that the C ABI in vlb3d.hip calls.
#define VLB3_PART 2
#include "vlb3d.hip"
