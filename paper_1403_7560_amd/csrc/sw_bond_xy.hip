// sw_bond_xy.hip -- XY instantiations of the bond and flip kernels.
#include "sw_bond.h"

namespace swmc {

hipError_t launch_bond_xy(int dim, int v, const InstDesc *dd, const int2 *tm, int nt, int nf, uint32_t k,
                          int mode, hipStream_t s, hipEvent_t t0, hipEvent_t t1)
{
    return dim == 2 ? bond_dispatch<XY, 2>(v, dd, tm, nt, nf, k, mode, s, t0, t1)
                    : bond_dispatch<XY, 3>(v, dd, tm, nt, nf, k, mode, s, t0, t1);
}

hipError_t launch_flip_xy(int dim, int v, const InstDesc *dd, const int2 *tm, int nt, uint32_t k,
                          hipStream_t s)
{
    return dim == 2 ? flip_dispatch<XY, 2>(v, dd, tm, nt, k, s) : flip_dispatch<XY, 3>(v, dd, tm, nt, k, s);
}

}  // namespace swmc
