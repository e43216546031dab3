// Launch code of the FP64 mode (see ops_impl.hpp).
#include "ops_impl.hpp"

template struct qap::Ops<qap::kPrecF64>;
