// Pass kernels, single precision, variant 2.
#include "fsa_launch.hpp"

template struct fsa::LaunchV<float, 2>;
