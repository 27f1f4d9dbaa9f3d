// F64 instantiation of the Ls-vectorised hop (one translation unit per
// storage precision so the kernels compile in parallel).
#include "hop_impl.h"

namespace mspcg {

template int launch_hop<F64>(const HopArgs<F64>&, int, int, bool, hipStream_t);
template long hop_grid_x<F64>(long, int);
template int launch_multi_hop<F64>(const MultiHop<F64>*, long, int, bool, bool, bool,
                                    bool, hipStream_t);

}  // namespace mspcg
