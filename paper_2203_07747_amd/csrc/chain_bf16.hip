// Layer-chain kernels instantiated for bf16 operands.
#include "chain_kernels.h"

namespace rtn {

template hipError_t chain_forward<P_BF16>(int, const ChainCfg&, const NetView&, int, const float*, const float*,
                                        const float*, void*, float*, float*, float*, hipStream_t);
template hipError_t chain_reverse<P_BF16>(int, const ChainCfg&, const NetView&, int, const void*, float*, float*,
                                        hipStream_t);
template hipError_t chain_geom<P_BF16>(int, int, int, int, ChainGeom*);

}  // namespace rtn
