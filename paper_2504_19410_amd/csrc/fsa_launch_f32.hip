// FP32 instantiation of the pass launchers.
#include "fsa_launch.hpp"

template struct fsa::Launch<float>;
