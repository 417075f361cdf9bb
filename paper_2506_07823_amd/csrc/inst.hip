// inst.hip -- explicit instantiation of the launch sequences for one padded
// order class and one storage type; compiled once per pair with
// -DLQR_TS=<tile size> -DLQR_S=<float|double>.
#include "runs.hpp"

#ifndef LQR_TS
#error "define LQR_TS"
#endif
#ifndef LQR_S
#error "define LQR_S"
#endif

namespace lqr {
LQR_DEFINE_RUNS(LQR_TS, LQR_S)
}  // namespace lqr
