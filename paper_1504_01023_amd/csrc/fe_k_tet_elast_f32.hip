// Tetrahedron, 3-component elasticity: kernel instantiations (float).
#include "fe_register.h"

namespace {
using namespace fe;
typedef float T;

int register_all()
{
#define BASE(MODE) reg_tet_elastic<T, MODE, 0, 1, 1, 1>(); reg_tet_elastic<T, MODE, 1, 1, 1, 1>();
    BASE(M_UNIFORM) BASE(M_ELEM) BASE(M_QP) BASE(M_ELEM_MIXED) BASE(M_QP_MIXED)
#undef BASE
#define TUNE(MODE, PK) \
    reg_tet_elastic<T, MODE, PK, 2, 1, 1>(); reg_tet_elastic<T, MODE, PK, 4, 1>(); \
    reg_tet_elastic<T, MODE, PK, 1, 0>(); reg_tet_elastic<T, MODE, PK, 2, 0>(); \
    reg_tet_elastic<T, MODE, PK, 1, 2>(); reg_tet_elastic<T, MODE, PK, 2, 2>();
    TUNE(M_ELEM, 1) TUNE(M_ELEM, 0) TUNE(M_UNIFORM, 1)
#undef TUNE
    return 0;
}
const int registered = register_all();
}  // namespace
