// Kernels of the D2Q5, the d velocity sets (Remark IV), every storage.
#include "mdf_kernels.h"

namespace mdf {

const LatOps &lat_ops_d2q5v()
{
    static const LatOps ops = make_lat_ops<LatD2Q5V>();
    return ops;
}

}  // namespace mdf
