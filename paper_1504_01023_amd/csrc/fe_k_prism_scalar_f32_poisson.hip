// Prism, scalar problem: kernel instantiations (float, TS_POISSON).
#include "fe_register.h"

namespace {
using namespace fe;
typedef float T;
constexpr int TS = TS_POISSON;

int register_all()
{
    // every coefficient mode and K format with a runtime point loop
#define BASE(MODE) \
    reg_prism_scalar<T, TS, MODE, 0, 0, 1, REF_KARG, 1>(); reg_prism_scalar<T, TS, MODE, 1, 0, 1, REF_KARG, 1>();
    BASE(M_UNIFORM) BASE(M_ELEM) BASE(M_QP) BASE(M_ELEM_MIXED) BASE(M_QP_MIXED) BASE(M_FUNC)
#undef BASE
    // tuning variants of the runtime point loop: cache policy and LDS
    // staging of the reference tables
#define TUNE(MODE, PK) \
    reg_prism_scalar<T, TS, MODE, PK, 0, 0, REF_KARG>(); reg_prism_scalar<T, TS, MODE, PK, 0, 1, REF_LDS>(); \
    reg_prism_scalar<T, TS, MODE, PK, 0, 0, REF_LDS>(); reg_prism_scalar<T, TS, MODE, PK, 0, 2, REF_KARG>();
    TUNE(M_QP, 0) TUNE(M_ELEM, 0) TUNE(M_UNIFORM, 1) TUNE(M_UNIFORM, 0) TUNE(M_FUNC, 0)
#undef TUNE
    // the SQS and SSQ loop orders, for the order comparison (the paper's
    // "Poisson": per-point right-hand side; "conv-diff": element constants)
#define ORDERS(MODE) \
    reg_prism_scalar_order<T, TS, MODE, 0, ORDER_SQS, 1>(); reg_prism_scalar_order<T, TS, MODE, 0, ORDER_SSQ, 1>(); \
    reg_prism_scalar_order<T, TS, MODE, 0, ORDER_SQS, 0>(); reg_prism_scalar_order<T, TS, MODE, 0, ORDER_SSQ, 0>();
    ORDERS(M_QP_MIXED) ORDERS(M_ELEM) ORDERS(M_QP)
#undef ORDERS
    // symmetric problems asked for full K: upper triangle accumulated
#define SYMFULL(MODE) \
    reg_prism_scalar<T, TS, MODE, 2, 0, 1, REF_KARG, 1>(); reg_prism_scalar<T, TS, MODE, 2, 0, 0, REF_KARG>(); \
    reg_prism_scalar<T, TS, MODE, 2, 0, 2, REF_KARG>(); reg_prism_scalar<T, TS, MODE, 2, 0, 1, REF_LDS>();
    SYMFULL(M_UNIFORM) SYMFULL(M_QP_MIXED) SYMFULL(M_ELEM_MIXED)
#undef SYMFULL
    // the points of an element split over 2, 3 or 6 lanes
#define LANES(MODE) \
    reg_prism_scalar_lanes<T, TS, MODE, 0, 2, 1, REF_KARG>(); \
    reg_prism_scalar_lanes<T, TS, MODE, 0, 3, 1, REF_KARG>(); \
    reg_prism_scalar_lanes<T, TS, MODE, 0, 6, 1, REF_KARG>();
    LANES(M_QP_MIXED)
#undef LANES
    return 0;
}
const int registered = register_all();
}  // namespace
