// dugks2p_fused.hpp -- fused one-kernel time step (placeholder until written).
#pragma once
#include "dugks2p_dev.hpp"

namespace dg {
struct FusedPlan {
  int ok;
};
inline FusedPlan make_fused_plan(const Consts &, int) { return FusedPlan{0}; }
template <class T>
inline void fused_step(const FusedPlan &, const Consts &, const T *, T *, hipStream_t,
                       hipError_t &err) {
  err = hipErrorNotSupported;
}
}  // namespace dg
