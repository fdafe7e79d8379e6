// Kernels of the D2Q4, the d velocity sets (Remark IV), every storage.
#include "mdf_kernels.h"

namespace mdf {

const LatOps &lat_ops_d2q4v()
{
    static const LatOps ops = make_lat_ops<LatD2Q4V>();
    return ops;
}

}  // namespace mdf
