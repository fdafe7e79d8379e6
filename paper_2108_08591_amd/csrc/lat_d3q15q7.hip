// Kernels of the lattice per set: D3Q15 velocity sets with the set a = 0 on D3Q7, every storage.
#include "mdf_kernels.h"

namespace mdf {

const LatOps &lat_ops_d3q15q7()
{
    static const LatOps ops = make_lat_ops<LatD3Q15Q7>();
    return ops;
}

}  // namespace mdf
