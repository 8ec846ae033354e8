// complex64 instances of the reg DFT schedule (k_lfft_impl.h).
#include "k_lfft_impl.h"

namespace mr1l {

int reg_launch_f(Plan &p, int N, const int32_t *d_lats, int nl, const MDesc *d_md, const void *in, void *out,
                 double theta, uint32_t *bitmap, int mode, double scale, int by_m)
{
    return reg_launch_t<float>(p, N, d_lats, nl, d_md, in, out, theta, bitmap, mode, scale, by_m);
}

int lfft_attrs_f() { return reg_attrs_t<float>(); }

}  // namespace mr1l
