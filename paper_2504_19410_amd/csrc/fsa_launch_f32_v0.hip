// Pass kernels, single precision, variant 0.
#include "fsa_launch.hpp"

template struct fsa::LaunchV<float, 0>;
