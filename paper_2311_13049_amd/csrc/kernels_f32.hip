// FP32 instantiations of the launchers (transforms and pointwise work in
// float; expansion coefficients, multipliers, propagator and state in double;
// forward transforms of caller data in double).
#include "launch_impl.hpp"

namespace vofl {
template struct Launch<float>;
template hipError_t Launch<float>::contig<float>(int, const ContigArgs<float, float>&, int, hipStream_t, int);
template hipError_t Launch<float>::contig<double>(int, const ContigArgs<float, double>&, int, hipStream_t, int);
}
