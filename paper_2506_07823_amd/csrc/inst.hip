// inst.hip -- explicit instantiation of the launch sequences for one padded
// order class; compiled once per class with -DLQR_TS=<tile size>.
#include "runs.hpp"

#ifndef LQR_TS
#error "define LQR_TS"
#endif

namespace lqr {
LQR_DEFINE_RUNS(LQR_TS)
}  // namespace lqr
