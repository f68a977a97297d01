// FP32 instances of the streaming kernels (B up to 256 seeds per block).
#include <algorithm>
#include <type_traits>
#define MAR_T float
#define MAR_DISPATCH_BIG(...)                                         \
    if (B == 256) { constexpr int BB = 256; __VA_ARGS__; }
#include "mar_launch_impl.h"
