// Kernels of the D3Q6, the d velocity sets (Remark IV), every storage.
#include "mdf_kernels.h"

namespace mdf {

const LatOps &lat_ops_d3q6v()
{
    static const LatOps ops = make_lat_ops<LatD3Q6V>();
    return ops;
}

}  // namespace mdf
