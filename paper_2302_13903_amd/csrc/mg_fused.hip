// mg_fused.hip -- fused multi-sweep smoothing kernels (large levels).
#include "mg_fused.h"

namespace mg {

template <typename T>
bool fused_supported(int) {
  return false;
}

template <typename T>
void launch_fused_smooth(T*, const T*, int, double, double, int, const LevelBC&, hipStream_t) {}

template <typename T>
std::string fused_smooth_name(int, int) {
  return "none";
}

template <typename T>
double fused_smooth_bytes(int, int) {
  return 0.0;
}

template bool fused_supported<double>(int);
template bool fused_supported<float>(int);
template void launch_fused_smooth<double>(double*, const double*, int, double, double, int, const LevelBC&, hipStream_t);
template void launch_fused_smooth<float>(float*, const float*, int, double, double, int, const LevelBC&, hipStream_t);
template std::string fused_smooth_name<double>(int, int);
template std::string fused_smooth_name<float>(int, int);
template double fused_smooth_bytes<double>(int, int);
template double fused_smooth_bytes<float>(int, int);

}  // namespace mg
