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
    reg_prism_elastic<T, MODE, PK, 0, 0, REF_KARG>(); reg_prism_elastic<T, MODE, PK, 0, 1, REF_LDS>(); \
    reg_prism_elastic<T, MODE, PK, 0, 2, REF_KARG>();
    TUNE(M_ELEM, 1) TUNE(M_ELEM, 0)
#undef TUNE
    // two or three passes over the points, rows of K split (fewer live accumulators)
#define SPLIT2(MODE, PK) \
    reg_prism_elastic<T, MODE, PK, 0, 1, REF_KARG, 1, 2>(); reg_prism_elastic<T, MODE, PK, 0, 0, REF_KARG, 0, 2>(); \
    reg_prism_elastic<T, MODE, PK, 0, 1, REF_LDS, 0, 2>(); reg_prism_elastic<T, MODE, PK, 0, 2, REF_KARG, 0, 2>();
    SPLIT2(M_ELEM, 1) SPLIT2(M_ELEM, 0) SPLIT2(M_UNIFORM, 1) SPLIT2(M_ELEM_MIXED, 1)
#undef SPLIT2
#define SPLIT3(MODE, PK) \
    reg_prism_elastic<T, MODE, PK, 0, 1, REF_KARG, 1, 3>(); reg_prism_elastic<T, MODE, PK, 0, 0, REF_KARG, 0, 3>();
    SPLIT3(M_ELEM, 1) SPLIT3(M_ELEM, 0)
#undef SPLIT3
    return 0;
}
const int registered = register_all();
}  // namespace
