// Launch code of the FP32 certified (rounded toward -inf) mode (see ops_impl.hpp).
#include "ops_impl.hpp"

template struct qap::Ops<qap::kPrecF32Down>;
