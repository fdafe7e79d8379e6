// Kernels of the D3Q6, all d + 1 sets, every storage.
#include "mdf_kernels.h"

namespace mdf {

const LatOps &lat_ops_d3q6()
{
    static const LatOps ops = make_lat_ops<LatD3Q6>();
    return ops;
}

}  // namespace mdf
