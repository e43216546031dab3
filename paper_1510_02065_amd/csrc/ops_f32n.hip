// Launch code of the FP32 round-to-nearest mode (see ops_impl.hpp).
#include "ops_impl.hpp"

template struct qap::Ops<qap::kPrecF32Near>;
