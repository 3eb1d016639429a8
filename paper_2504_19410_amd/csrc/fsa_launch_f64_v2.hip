// Pass kernels, double precision, variant 2.
#include "fsa_launch.hpp"

template struct fsa::LaunchV<double, 2>;
