// Kernels of the lattice per set: D2Q9 velocity sets with the set a = 0 on D2Q5, every storage.
#include "mdf_kernels.h"

namespace mdf {

const LatOps &lat_ops_d2q9q5()
{
    static const LatOps ops = make_lat_ops<LatD2Q9Q5>();
    return ops;
}

}  // namespace mdf
