// Kernels of the D2Q9, all d + 1 sets, every storage.
#include "mdf_kernels.h"

namespace mdf {

const LatOps &lat_ops_d2q9()
{
    static const LatOps ops = make_lat_ops<LatD2Q9>();
    return ops;
}

}  // namespace mdf
