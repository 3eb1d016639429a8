// Pass kernels, double precision, variant 1.
#include "fsa_launch.hpp"

template struct fsa::LaunchV<double, 1>;
