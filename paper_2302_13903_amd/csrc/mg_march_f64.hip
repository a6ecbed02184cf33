// mg_march_f64.hip -- the two-sweep streaming passes (mg_march.inl) instantiated in FP64.
#define MG_MARCH_T double
#include "mg_march.inl"
