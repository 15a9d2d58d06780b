// Tetrahedron, scalar problem: kernel instantiations (double, TS_POISSON).
#include "fe_register.h"

namespace {
using namespace fe;
typedef double T;
constexpr int TS = TS_POISSON;

int register_all()
{
    // every coefficient mode and K format, base variant (1 element per
    // lane, non-temporal), plain and batched forms
#define BASE(MODE) reg_tet_scalar<T, TS, MODE, 0, 1, 1, 1>(); reg_tet_scalar<T, TS, MODE, 1, 1, 1, 1>();
    BASE(M_UNIFORM) BASE(M_ELEM) BASE(M_QP) BASE(M_ELEM_MIXED) BASE(M_QP_MIXED) BASE(M_FUNC)
#undef BASE
    reg_tet_scalar<T, TS, M_FUNC, 0, 2, 1>();
    reg_tet_scalar<T, TS, M_FUNC, 0, 2, 0>();
    // tuning variants: elements per lane and cache policy (default,
    // streaming, streaming stores only)
#define TUNE(MODE, PK) \
    reg_tet_scalar<T, TS, MODE, PK, 2, 1, 1>(); reg_tet_scalar<T, TS, MODE, PK, 4, 1>(); \
    reg_tet_scalar<T, TS, MODE, PK, 1, 0>(); reg_tet_scalar<T, TS, MODE, PK, 2, 0, 1>(); \
    reg_tet_scalar<T, TS, MODE, PK, 4, 0>(); \
    reg_tet_scalar<T, TS, MODE, PK, 1, 2>(); reg_tet_scalar<T, TS, MODE, PK, 2, 2>(); \
    reg_tet_scalar<T, TS, MODE, PK, 4, 2>();
    TUNE(M_UNIFORM, 1) TUNE(M_UNIFORM, 0) TUNE(M_ELEM, 0) TUNE(M_ELEM, 1) TUNE(M_QP, 0)
#undef TUNE
    reg_tet_scalar<T, TS, M_QP_MIXED, 0, 2, 1>();
    reg_tet_scalar<T, TS, M_QP_MIXED, 0, 2, 0>();
    reg_tet_scalar<T, TS, M_QP_MIXED, 0, 1, 0>();
    reg_tet_scalar<T, TS, M_ELEM_MIXED, 0, 2, 1>();
    reg_tet_scalar<T, TS, M_ELEM_MIXED, 1, 2, 1>();
    return 0;
}
const int registered = register_all();
}  // namespace
