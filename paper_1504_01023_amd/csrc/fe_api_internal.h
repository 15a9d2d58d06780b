// fe_api_internal.h -- host-side helpers shared by the C-ABI translation
// units (dispatcher, tuner, batcher). Not part of the public ABI.
#pragma once

#include "fe.h"
#include "fe_internal.h"

namespace fe {

// A validated, fully resolved launch.
struct Plan {
    KArgs args;
    const KernelEntry *entry = nullptr;
    unsigned grid = 0, block = 0;
    KernelKey key{};
    fe_variant variant{};
};

int fail(int status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

// form: 0 = plain launch (coordinates per element), 1 = indexed geometry
// (coordinates gathered through connectivity; `coords` is ignored and the
// element-group alignment applies to the connectivity array instead).
int plan(const fe_problem *problem, int elem, int64_t n_elem, const double *coords,
         const void *coeffs, int64_t ld_in, const fe_quad_rule *rule, void *out_K, void *out_F,
         int64_t ld_out, const fe_variant *variant, Plan &pl, int form = 0,
         const int32_t *conn = nullptr, int64_t ld_conn = 0);
int launch(const Plan &pl, hipStream_t stream);
void fill_reference(int elem, const fe_quad_rule &rule, KArgs &a);
// NULL rule, point count outside 1..FE_MAX_QP, non-finite points or weights
int check_rule(const fe_quad_rule *r);

// Tuning table: variant per (kernel family, point count).
int tuning_lookup(const KernelKey &family, int n_q, fe_variant &out);

// Persistent batched launches (fe_batch.cpp): the resolved plan of kind k
// (its grid and the chunk size set), the validation of one request of that
// kind (*wide: its rows and pointers suit the kind's elements per lane), and
// chunk c of a request.
int batch_kind_plan(const fe_batch_kind &bk, int k, int64_t chunk_elems, int blocks_per_kind,
                    Plan &out);
int batch_check_request(const Plan &pl, int kind, int64_t n_elem, const double *coords,
                        const void *coeffs, int64_t ld_in, const void *out_K, const void *out_F,
                        int64_t ld_out, bool *wide);
Chunk batch_chunk(int64_t c, int64_t chunk_elems, int64_t n_elem, const double *coords,
                  const void *coeffs, int64_t ld_in, void *out_K, void *out_F, int64_t ld_out,
                  bool wide);

}  // namespace fe
