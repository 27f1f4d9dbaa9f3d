// F16 instantiation of the Ls-vectorised hop (one translation unit per
// storage precision so the kernels compile in parallel).
#include "hop_impl.h"

namespace mspcg {

template int launch_hop<F16>(const HopArgs<F16>&, int, int, bool, hipStream_t);

bool multi_hop_ls(int Ls) { return Ls == 8 || Ls == 12 || Ls == 16; }
template long hop_grid_x<F16>(long, int);
template int launch_multi_hop<F16>(const MultiHop<F16>*, long, int, bool, bool, bool,
                                    bool, hipStream_t);

}  // namespace mspcg
