// Pass kernels, single precision, variant 4.
#include "fsa_launch.hpp"

template struct fsa::LaunchV<float, 4>;
