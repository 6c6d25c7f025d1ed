// FP32 instantiations of the launchers (transforms and pointwise work in
// float; expansion coefficients, multipliers, propagator and state in double).
#include "launch_impl.hpp"

namespace vofl {
template struct Launch<float>;
}
