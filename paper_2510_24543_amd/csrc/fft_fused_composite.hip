// The direction write fused with the line search's first z pass for the
// composite preconditioner P_Delta^-1 P_V^-1 (zmode 2; arXiv:2510.24543,
// Sec. IV.B Eq. (18), Sec. IV.C, Sec. V): its instantiations, in a translation
// unit of their own so that they compile beside those for P_V.
#include "fft_dirwrite.h"

namespace bec {

hipError_t fft_dirwrite_z_pass_composite(int L, int variant, const FftPassArgs& Z, const PwParams& P,
                                         const DirArgs& A, hipStream_t st)
{
    return dirwrite_z_launch<2>(L, variant, Z, P, A, st);
}

}  // namespace bec
