// Prism, general 3-component CDR: kernel instantiations (double).
#include "fe_register.h"

namespace {
using namespace fe;
typedef double T;

int register_all()
{
    // runtime point loop; cache policy and LDS staging of the reference tables
#define VARIANTS(MODE) \
    reg_prism_vector<T, MODE, 0, 1, REF_KARG>(); reg_prism_vector<T, MODE, 0, 0, REF_KARG>(); \
    reg_prism_vector<T, MODE, 0, 1, REF_LDS>();
    VARIANTS(M_ELEM) VARIANTS(M_QP)
#undef VARIANTS
    return 0;
}
const int registered = register_all();
}  // namespace
