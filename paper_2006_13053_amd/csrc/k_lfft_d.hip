// complex128 instances of the reg and split DFT schedules (k_lfft_impl.h).
#include "k_lfft_impl.h"

namespace mr1l {

int reg_launch_d(Plan &p, int N, const int32_t *d_lats, int nl, const MDesc *d_md, const void *in, void *out,
                 double theta, uint32_t *bitmap, int mode, double scale, int by_m)
{
    return reg_launch_t<double>(p, N, d_lats, nl, d_md, in, out, theta, bitmap, mode, scale, by_m);
}

int split_launch_d(Plan &p, int K, const int32_t *d_lats, int nl, const MDesc *d_md, const void *in, void *out,
                   double theta, uint32_t *bitmap, int mode, double scale, int by_m)
{
    return split_launch_t<double>(p, K, d_lats, nl, d_md, in, out, theta, bitmap, mode, scale, by_m);
}

int lfft_attrs_d()
{
    const int rc = reg_attrs_t<double>();
    return rc ? rc : split_attrs_t<double>();
}

}  // namespace mr1l
