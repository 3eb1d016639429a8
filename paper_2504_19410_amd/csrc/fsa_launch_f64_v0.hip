// Pass kernels, double precision, variant 0.
#include "fsa_launch.hpp"

template struct fsa::LaunchV<double, 0>;
