// Kernels of the D2Q9, the d velocity sets (Remark IV), every storage.
#include "mdf_kernels.h"

namespace mdf {

const LatOps &lat_ops_d2q9v()
{
    static const LatOps ops = make_lat_ops<LatD2Q9V>();
    return ops;
}

}  // namespace mdf
