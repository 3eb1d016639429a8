// Pass kernels, double precision, variant 4.
#include "fsa_launch.hpp"

template struct fsa::LaunchV<double, 4>;
