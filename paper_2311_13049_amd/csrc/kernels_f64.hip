// FP64 instantiations of the launchers.
#include "launch_impl.hpp"

namespace vofl {
template struct Launch<double>;
template hipError_t Launch<double>::contig<double>(int, const ContigArgs<double, double>&, int, hipStream_t, int);
}
