// mg_march_f32.hip -- the two-sweep streaming passes (mg_march.inl) instantiated in FP32, the
// precision of the inner cycles of mixed-precision solves.
#define MG_MARCH_T float
#include "mg_march.inl"
