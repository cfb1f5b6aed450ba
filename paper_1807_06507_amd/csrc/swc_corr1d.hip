// 1-D sliding-window correlation.  Provisional path: a length-N series is
// the 1 x N image of the fused 2-D kernel (window 1 x k, step 1 x s).
#include "swc_device.hpp"
#include "swc_internal.h"

namespace swc {

static swc_problem as_2d(const swc_problem& p)
{
    swc_problem q = p;
    q.ndim = 2;
    q.shape[0] = 1;
    q.shape[1] = p.shape[0];
    q.window[0] = 1;
    q.window[1] = p.window[0];
    q.step[0] = 1;
    q.step[1] = p.step[0];
    return q;
}

bool cfg_ok_1d(const swc_problem& p, const LaunchCfg& L)
{
    LaunchCfg L2 = L;
    L2.TH = 1;
    return cfg_ok_2d(as_2d(p), L2);
}

hipError_t launch_corr1d(const swc_problem& p, const int64_t* oshape, const LaunchCfg& L,
                         const void* x, const void* y, float* c, uint8_t* flags,
                         hipStream_t s, int force)
{
    swc_problem q = as_2d(p);
    int64_t o2[3] = {1, oshape[0], 1};
    LaunchCfg L2 = L;
    L2.TH = 1;
    return launch_corr2d(q, o2, L2, x, y, c, flags, s, force);
}

}  // namespace swc
