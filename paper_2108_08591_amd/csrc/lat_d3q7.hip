// Kernels of the D3Q7, all d + 1 sets, every storage.
#include "mdf_kernels.h"

namespace mdf {

const LatOps &lat_ops_d3q7()
{
    static const LatOps ops = make_lat_ops<LatD3Q7>();
    return ops;
}

}  // namespace mdf
