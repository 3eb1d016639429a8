// Pass kernels, single precision, variant 1.
#include "fsa_launch.hpp"

template struct fsa::LaunchV<float, 1>;
