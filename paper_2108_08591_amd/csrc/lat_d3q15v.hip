// Kernels of the D3Q15, the d velocity sets (Remark IV), every storage.
#include "mdf_kernels.h"

namespace mdf {

const LatOps &lat_ops_d3q15v()
{
    static const LatOps ops = make_lat_ops<LatD3Q15V>();
    return ops;
}

}  // namespace mdf
