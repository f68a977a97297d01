// FP64 instances of the streaming kernels (B up to 128 seeds per block).
#include <algorithm>
#include <type_traits>
#define MAR_T double
#define MAR_DISPATCH_BIG(...) \
    do {                      \
    } while (0)
#include "mar_launch_impl.h"
