// fe_register.h -- registration helpers for the kernel translation units.
#pragma once

#include <type_traits>

#include "fe_device.h"

namespace fe {

// Registers the plain kernel; B = 1 also registers the batched (persistent)
// form and the indexed-geometry form. The consumer form (ap: matrix-free
// application and assembly) and the natural-order form (ao) are registered
// as given.
template <class P, int V, int NT, int REF, int B = 0>
inline void reg(int elem, int kind, int prec, int terms, int mode, int packed, int nq, int split = 1,
                int order = 1, ApplyLaunchFn ap = nullptr, AosLaunchFn ao = nullptr)
{
    KernelKey k{elem, kind, prec, terms, mode, packed, V, NT, REF, nq, split, order, 1};
    BatchLaunchFn bl = nullptr;
    IdxLaunchFn il = nullptr;
    if constexpr (B != 0) {
        bl = &launch_fe_batch_kernel<P, V, NT, REF>;
        il = &launch_fe_kernel_idx<P, V, NT, REF>;
    }
    register_kernel(KernelEntry{k, &launch_fe_kernel<P, V, NT, REF>,
                                reinterpret_cast<const void *>(&fe_kernel<P, V, NT, REF>), bl,
                                il, ap, ao});
}

// The natural-order form of a problem class with NV vertices, for the base
// variants (one element per lane, with the batched and indexed forms).
template <class P, int NV, int V, int NT, int REF, int B>
constexpr AosLaunchFn aos_form()
{
    if constexpr (V == 1 && B != 0)
        return &launch_fe_kernel_aos<P, NV, NT, REF>;
    else
        return nullptr;
}

// The matrix-free form of a problem class with NV vertices and NC
// components, for the base variants (one element per lane, with the batched
// and indexed forms).
template <class P, int NV, int NC, typename T, int V, int NT, int REF, int B>
constexpr ApplyLaunchFn apply_form()
{
    if constexpr (V == 1 && B != 0)
        return &launch_fe_apply<P, NV, NC, T, NT, REF>;
    else
        return nullptr;
}

template <typename T>
constexpr int prec_of() { return std::is_same<T, float>::value ? FE_FP32_BULK : FE_FP64; }

template <typename T, int TERMS, int MODE, int PK, int V, int NT, int B = 0>
inline void reg_tet_scalar()
{
    typedef TetScalar<T, TERMS, MODE, PK> P;
    reg<P, V, NT, REF_KARG, B>(FE_TET4, FE_SCALAR_CDR, prec_of<T>(), TERMS, MODE, PK, 0, 1, 1,
                               apply_form<P, 4, 1, T, V, NT, REF_KARG, B>(),
                               aos_form<P, 4, V, NT, REF_KARG, B>());
}

template <typename T, int MODE, int PK, int V, int NT, int B = 0>
inline void reg_tet_elastic()
{
    typedef TetElastic<T, MODE, PK> P;
    reg<P, V, NT, REF_KARG, B>(FE_TET4, FE_ELASTICITY, prec_of<T>(), TS_ELAST, MODE, PK, 0, 1, 1,
                               apply_form<P, 4, 3, T, V, NT, REF_KARG, B>(),
                               aos_form<P, 4, V, NT, REF_KARG, B>());
}

template <typename T, int TERMS, int MODE, int PK, int NQ, int NT, int REF, int B = 0>
inline void reg_prism_scalar()
{
    typedef PrismScalar<T, TERMS, MODE, PK, NQ> P;
    reg<P, 1, NT, REF, B>(FE_PRISM6, FE_SCALAR_CDR, prec_of<T>(), TERMS, MODE, PK, NQ, 1, 1,
                          apply_form<P, 6, 1, T, 1, NT, REF, B>(), aos_form<P, 6, 1, NT, REF, B>());
}

// Prism scalar QSS kernels with the points of an element split between G
// lanes (plain form only).
template <typename T, int TERMS, int MODE, int PK, int G, int NT, int REF>
inline void reg_prism_scalar_lanes()
{
    typedef PrismScalar<T, TERMS, MODE, PK, 0> P;
    KernelKey k{FE_PRISM6, FE_SCALAR_CDR, prec_of<T>(), TERMS, MODE, PK, 1, NT, REF, 0, 1, 1, G};
    register_kernel(KernelEntry{k, &launch_fe_kernel_lanes<P, G, NT, REF>,
                                reinterpret_cast<const void *>(&fe_kernel_lanes<P, G, NT, REF>),
                                nullptr, nullptr, nullptr, nullptr});
}

// Prism scalar kernels in the SQS / SSQ loop orders (one element per lane).
template <typename T, int TERMS, int MODE, int PK, int ORDER, int NT>
inline void reg_prism_scalar_order()
{
    reg<PrismScalarOrder<T, TERMS, MODE, PK, ORDER>, 1, NT, REF_KARG>(
        FE_PRISM6, FE_SCALAR_CDR, prec_of<T>(), TERMS, MODE, PK, 0, 1, ORDER);
}

template <typename T, int MODE, int PK, int NQ, int NT, int REF, int B = 0, int SPLIT = 1>
inline void reg_prism_elastic()
{
    typedef PrismElastic<T, MODE, PK, NQ, SPLIT> P;
    reg<P, 1, NT, REF, B>(FE_PRISM6, FE_ELASTICITY, prec_of<T>(), TS_ELAST, MODE, PK, NQ, SPLIT, 1,
                          apply_form<P, 6, 3, T, 1, NT, REF, B>(), aos_form<P, 6, 1, NT, REF, B>());
}

// General 3-component CDR (coefficients per element or per point, full K).
// (batched, indexed, consumer and natural-order forms for the streaming
// one-element-per-lane variants)
template <typename T, int MODE, int V, int NT>
inline void reg_tet_vector()
{
    typedef TetVector<T, MODE> P;
    reg<P, V, NT, REF_KARG, V == 1 && NT == 1>(FE_TET4, FE_VECTOR_CDR, prec_of<T>(), TS_FULL, MODE, 0,
                                              0, 1, 1,
                            apply_form<P, 4, 3, T, V, NT, REF_KARG, V == 1 && NT == 1>(),
                            aos_form<P, 4, V, NT, REF_KARG, V == 1 && NT == 1>());
}

template <typename T, int MODE, int NQ, int NT, int REF>
inline void reg_prism_vector()
{
    typedef PrismVector<T, MODE, NQ> P;
    reg<P, 1, NT, REF, NT == 1 && REF == REF_KARG>(FE_PRISM6, FE_VECTOR_CDR, prec_of<T>(), TS_FULL,
                                                   MODE, 0, NQ, 1, 1,
                       apply_form<P, 6, 3, T, 1, NT, REF, NT == 1 && REF == REF_KARG>(),
                       aos_form<P, 6, 1, NT, REF, NT == 1 && REF == REF_KARG>());
}

}  // namespace fe
