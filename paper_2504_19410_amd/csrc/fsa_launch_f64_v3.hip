// Pass kernels, double precision, variant 3.
#include "fsa_launch.hpp"

template struct fsa::LaunchV<double, 3>;
