// Tetrahedron, general 3-component CDR: kernel instantiations (float).
#include "fe_register.h"

namespace {
using namespace fe;
typedef float T;

int register_all()
{
    // per-element coefficients: 1 or 2 elements per lane, streaming or
    // default cache policy; per-point coefficients one element per lane (two
    // exceed the register file)
    reg_tet_vector<T, M_ELEM, 1, 1>(); reg_tet_vector<T, M_ELEM, 2, 1>();
    reg_tet_vector<T, M_ELEM, 1, 0>(); reg_tet_vector<T, M_ELEM, 2, 0>();
    reg_tet_vector<T, M_ELEM, 1, 2>(); reg_tet_vector<T, M_ELEM, 2, 2>();
    reg_tet_vector<T, M_QP, 1, 1>(); reg_tet_vector<T, M_QP, 1, 0>();
    return 0;
}
const int registered = register_all();
}  // namespace
