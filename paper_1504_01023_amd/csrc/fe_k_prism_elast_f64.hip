// Prism, 3-component elasticity: kernel instantiations (double).
#include "fe_register.h"

namespace {
using namespace fe;
typedef double T;

int register_all()
{
#define BASE(MODE) \
    reg_prism_elastic<T, MODE, 0, 0, 1, REF_KARG, 1>(); reg_prism_elastic<T, MODE, 1, 0, 1, REF_KARG, 1>();
    BASE(M_UNIFORM) BASE(M_ELEM) BASE(M_QP) BASE(M_ELEM_MIXED) BASE(M_QP_MIXED)
#undef BASE
#define TUNE(MODE, PK) \
    reg_prism_elastic<T, MODE, PK, 0, 0, REF_KARG>(); reg_prism_elastic<T, MODE, PK, 0, 1, REF_LDS>();
    TUNE(M_ELEM, 1) TUNE(M_ELEM, 0)
#undef TUNE
    return 0;
}
const int registered = register_all();
}  // namespace
