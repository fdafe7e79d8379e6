// Kernels of the D3Q15, all d + 1 sets, every storage.
#include "mdf_kernels.h"

namespace mdf {

const LatOps &lat_ops_d3q15()
{
    static const LatOps ops = make_lat_ops<LatD3Q15>();
    return ops;
}

}  // namespace mdf
