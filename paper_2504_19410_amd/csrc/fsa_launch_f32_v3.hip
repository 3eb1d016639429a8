// Pass kernels, single precision, variant 3.
#include "fsa_launch.hpp"

template struct fsa::LaunchV<float, 3>;
