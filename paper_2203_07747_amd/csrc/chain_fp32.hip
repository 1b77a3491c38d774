// Layer-chain kernels instantiated for fp32 operands.
#include "chain_kernels.h"

namespace rtn {

template hipError_t chain_forward<P_FP32>(int, const ChainCfg&, const NetView&, int, const float*, const float*,
                                        const float*, void*, float*, float*, float*, hipStream_t);
template hipError_t chain_reverse<P_FP32>(int, const ChainCfg&, const NetView&, int, const void*, float*, float*,
                                        hipStream_t);
template hipError_t chain_geom<P_FP32>(int, int, int, int, ChainGeom*);

}  // namespace rtn
