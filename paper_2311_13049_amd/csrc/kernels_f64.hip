// FP64 instantiations of the launchers.
#include "launch_impl.hpp"

namespace vofl {
template struct Launch<double>;
}
