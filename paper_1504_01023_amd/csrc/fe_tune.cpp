// fe_tune.cpp -- parameter-based tuning by exhaustive search (the approach
// of Sec. 4.3: compile-time variants of one kernel, all run, the fastest
// kept), extended with the GPU launch shape. The table maps a kernel family
// (element, problem, precision, term set, coefficient mode, K format, point
// count) to the variant fe_integrate uses.
//
// Two tables: the caller's (fe_tuning_set, fe_tuning_load, fe_autotune) and
// the built-in one, the committed table measured on MI355X and compiled into
// the library. The built-in entries apply, for families the caller has not
// tuned, when the device the library first plans a launch on has the table's
// GPU architecture and the HIP runtime has the table's ROCm major version.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <tuple>
#include <vector>

#include "fe.h"
#include "fe_api_internal.h"

namespace fe {

typedef std::tuple<int, int, int, int, int, int, int> FamilyKey;

extern const char *const builtin_tuning_text;  // the committed table (build.py)

static std::mutex g_tune_mu;
static std::map<FamilyKey, fe_variant> &table()
{
    static std::map<FamilyKey, fe_variant> t;
    return t;
}

static FamilyKey family_of(const KernelKey &k, int n_q)
{
    return FamilyKey(k.elem, k.kind, k.prec, k.terms, k.mode, k.packed, n_q);
}

// One line of a table: 1 = an entry, 0 = blank or comment, -1 = malformed.
static int parse_line(const char *line, FamilyKey &key, fe_variant &v)
{
    while (*line == ' ' || *line == '\t')
        ++line;
    if (*line == '#' || *line == '\n' || *line == '\r' || *line == 0)
        return 0;
    int a[7];
    v = fe_variant{};
    const int got = std::sscanf(line, "%d %d %d %d %d %d %d | %d %d %d %d %d %d %d %d", &a[0], &a[1],
                                &a[2], &a[3], &a[4], &a[5], &a[6], &v.wg_size, &v.elems_per_thread,
                                &v.ref_in_lds, &v.nontemporal, &v.blocks, &v.row_split,
                                &v.loop_order, &v.lanes);
    // tables written before the row-split / loop-order / lanes fields
    if (got == 12)
        v.row_split = 1;
    if (got >= 12 && got <= 13)
        v.loop_order = 1;
    if (got >= 12 && got <= 14)
        v.lanes = 1;
    else if (got != 15)
        return -1;
    key = FamilyKey(a[0], a[1], a[2], a[3], a[4], a[5], a[6]);
    return 1;
}

struct Builtin {
    std::map<FamilyKey, fe_variant> entries;
    char arch[64] = "";        // the table's architecture ("# arch gfx950")
    int rocm_major = -1;       // the table's ROCm major version ("# rocm 7.2")
    char device_arch[64] = ""; // the device's, when it could be queried
    int runtime_major = -1;
    bool active = false;
};

static Builtin &builtin()
{
    static Builtin b;
    static std::once_flag once;
    std::call_once(once, [] {
        // the table text: header fields, then entries
        const char *p = builtin_tuning_text;
        std::map<FamilyKey, fe_variant> entries;
        while (p && *p) {
            const char *eol = std::strchr(p, '\n');
            const size_t len = eol ? (size_t)(eol - p) : std::strlen(p);
            char line[512];
            const size_t n = len < sizeof(line) - 1 ? len : sizeof(line) - 1;
            std::memcpy(line, p, n);
            line[n] = 0;
            int maj = 0, min = 0;
            char arch[64];
            if (std::sscanf(line, "# arch %63s", arch) == 1)
                std::snprintf(b.arch, sizeof(b.arch), "%s", arch);
            else if (std::sscanf(line, "# rocm %d.%d", &maj, &min) >= 1)
                b.rocm_major = maj;
            FamilyKey k;
            fe_variant v;
            if (parse_line(line, k, v) == 1)
                entries[k] = v;
            p = eol ? eol + 1 : nullptr;
        }
        // the device the library is first used on (a failed query leaves no
        // error behind for the caller; one pending before is kept)
        const hipError_t pending = hipPeekAtLastError();
        int dev = -1;
        hipDeviceProp_t prop;
        bool ok = hipGetDevice(&dev) == hipSuccess &&
                  hipGetDeviceProperties(&prop, dev) == hipSuccess;
        int rt = 0;
        ok = ok && hipRuntimeGetVersion(&rt) == hipSuccess;
        if (!ok) {
            if (pending == hipSuccess)
                (void)hipGetLastError();
            return;
        }
        std::snprintf(b.device_arch, sizeof(b.device_arch), "%s", prop.gcnArchName);
        char *colon = std::strchr(b.device_arch, ':');
        if (colon)
            *colon = 0;
        b.runtime_major = rt / 10000000;  // major * 10^7 + minor * 10^5 + patch
        if (std::strcmp(b.device_arch, b.arch) == 0 && b.runtime_major == b.rocm_major) {
            b.entries = entries;
            b.active = true;
        }
    });
    return b;
}

int tuning_lookup(const KernelKey &family, int n_q, fe_variant &out)
{
    const FamilyKey key = family_of(family, n_q);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = table().find(key);
        if (it != table().end()) {
            out = it->second;
            return FE_OK;
        }
    }
    const Builtin &b = builtin();
    auto it = b.entries.find(key);
    if (it == b.entries.end())
        return FE_ERR_INVALID_ARG;
    out = it->second;
    return FE_OK;
}

static int family_from_problem(const fe_problem *problem, fe_elem_type elem, int n_q, KernelKey &k)
{
    // Resolve the family by planning a zero-size launch with a dummy rule.
    double xi[3 * FE_MAX_QP] = {0}, w[FE_MAX_QP] = {0};
    if (n_q < 1 || n_q > FE_MAX_QP)
        return fail(FE_ERR_UNSUPPORTED, "n_q %d out of range", n_q);
    fe_quad_rule r{n_q, xi, w};
    Plan pl;
    const fe_variant base{256, 1, 2, 1, 0, 1, 1};
    int st = plan(problem, elem, 0, nullptr, nullptr, 0, &r, nullptr, nullptr, 0, &base, pl);
    if (st)
        return st;
    k = pl.key;
    return FE_OK;
}

}  // namespace fe

using namespace fe;

extern "C" {

int fe_tuning_get(const fe_problem *problem, fe_elem_type elem_type, int n_q, fe_variant *out)
{
    if (!out)
        return fail(FE_ERR_INVALID_ARG, "out is NULL");
    KernelKey k;
    int st = family_from_problem(problem, elem_type, n_q, k);
    if (st)
        return st;
    if (tuning_lookup(k, n_q, *out) != FE_OK)
        return fail(FE_ERR_INVALID_ARG, "no tuning entry for this problem");
    return FE_OK;
}

int fe_tuning_set(const fe_problem *problem, fe_elem_type elem_type, int n_q, const fe_variant *v)
{
    if (!v)
        return fail(FE_ERR_INVALID_ARG, "variant is NULL");
    KernelKey k;
    int st = family_from_problem(problem, elem_type, n_q, k);
    if (st)
        return st;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    table()[family_of(k, n_q)] = *v;
    return FE_OK;
}

int fe_tuning_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    table().clear();
    return FE_OK;
}

int fe_tuning_builtin(char *arch, int arch_len, int *n_entries)
{
    const Builtin &b = builtin();
    if (arch && arch_len > 0)
        std::snprintf(arch, (size_t)arch_len, "%s", b.arch);
    if (n_entries)
        *n_entries = b.active ? (int)b.entries.size() : 0;
    return b.active ? 1 : 0;
}

int fe_tuning_save(const char *path)
{
    if (!path)
        return fail(FE_ERR_INVALID_ARG, "path is NULL");
    FILE *f = std::fopen(path, "w");
    if (!f)
        return fail(FE_ERR_INVALID_ARG, "cannot open %s for writing", path);
    std::fprintf(f, "# libfe tuning table v4: elem kind prec terms mode packed n_q | wg vec ref nt blocks split order lanes\n");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &kv : table()) {
        const FamilyKey &k = kv.first;
        const fe_variant &v = kv.second;
        std::fprintf(f, "%d %d %d %d %d %d %d | %d %d %d %d %d %d %d %d\n", std::get<0>(k),
                     std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k), std::get<5>(k),
                     std::get<6>(k), v.wg_size, v.elems_per_thread, v.ref_in_lds, v.nontemporal,
                     v.blocks, v.row_split, v.loop_order, v.lanes ? v.lanes : 1);
    }
    std::fclose(f);
    return FE_OK;
}

int fe_tuning_load(const char *path)
{
    if (!path)
        return fail(FE_ERR_INVALID_ARG, "path is NULL");
    FILE *f = std::fopen(path, "r");
    if (!f)
        return fail(FE_ERR_INVALID_ARG, "cannot open %s", path);
    char line[512];
    std::map<FamilyKey, fe_variant> loaded;
    while (std::fgets(line, sizeof(line), f)) {
        FamilyKey k;
        fe_variant v;
        const int r = parse_line(line, k, v);
        if (r < 0) {
            std::fclose(f);
            return fail(FE_ERR_INVALID_ARG, "malformed tuning line: %s", line);
        }
        if (r == 1)
            loaded[k] = v;
    }
    std::fclose(f);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &kv : loaded)
        table()[kv.first] = kv.second;
    return FE_OK;
}

int fe_autotune(const fe_problem *problem, fe_elem_type elem_type, int64_t n_elem,
                const double *coords, const void *coeffs, int64_t ld_in,
                const fe_quad_rule *quad_rule, void *out_K, void *out_F, int64_t ld_out, int reps,
                fe_variant *best, double *best_ms, hipStream_t stream)
{
    if (reps < 1)
        reps = 1;
    // Validate the call once with the default variant.
    Plan base;
    int st = plan(problem, elem_type, n_elem, coords, coeffs, ld_in, quad_rule, out_K, out_F,
                  ld_out, nullptr, base);
    if (st)
        return st;
    if (n_elem == 0)
        return fail(FE_ERR_INVALID_ARG, "cannot tune on an empty batch");
    // Candidate variants: every compiled (vec, nt, ref, split) of this family,
    // times workgroup sizes and grid shapes (one group per lane, or a
    // persistent grid of 512..8192 workgroups).
    std::set<std::tuple<int, int, int, int, int, int>> shapes;
    for (int i = 0; i < kernel_count(); ++i) {
        const KernelKey &k = kernel_at(i)->key;
        if (k.elem == base.key.elem && k.kind == base.key.kind && k.prec == base.key.prec &&
            k.terms == base.key.terms && k.mode == base.key.mode && k.packed == base.key.packed &&
            (k.nq == quad_rule->n_q || k.nq == 0))
            shapes.insert(std::make_tuple(k.vec, k.nt, k.ref, k.split, k.order, k.lanes));
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(FE_ERR_HIP, "hipEventCreate failed");
    double best_t = 1e300;
    fe_variant best_v{};
    const int wgs[3] = {64, 128, 256};
    const int grids[6] = {0, 512, 1024, 2048, 4096, 8192};
    for (const auto &sh : shapes) {
        for (int wg : wgs) {
            for (int gb : grids) {
                const int ntk = std::get<1>(sh);  // kernel policy 0, 1, 2
                fe_variant v{wg, std::get<0>(sh), std::get<2>(sh) == REF_LDS ? 1 : 2,
                             ntk == 0 ? 2 : (ntk == 2 ? 3 : 1), gb, std::get<3>(sh),
                             std::get<4>(sh), std::get<5>(sh)};
                Plan pl;
                if (plan(problem, elem_type, n_elem, coords, coeffs, ld_in, quad_rule, out_K,
                         out_F, ld_out, &v, pl) != FE_OK)
                    continue;
                if (gb > 0 && (int64_t)gb >= (int64_t)pl.grid && gb != 0)
                    continue;  // same as the one-group-per-thread grid
                if (launch(pl, stream) != FE_OK)
                    continue;
                hipEventRecord(e0, stream);
                for (int r = 0; r < reps; ++r)
                    launch(pl, stream);
                hipEventRecord(e1, stream);
                if (hipEventSynchronize(e1) != hipSuccess) {
                    hipEventDestroy(e0);
                    hipEventDestroy(e1);
                    return fail(FE_ERR_HIP, "synchronisation failed while tuning");
                }
                float ms = 0.f;
                hipEventElapsedTime(&ms, e0, e1);
                const double t = ms / reps;
                if (t < best_t) {
                    best_t = t;
                    best_v = pl.variant;
                }
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (best_t >= 1e300)
        return fail(FE_ERR_UNSUPPORTED, "no variant could be launched");
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        table()[family_of(base.key, quad_rule->n_q)] = best_v;
    }
    if (best)
        *best = best_v;
    if (best_ms)
        *best_ms = best_t;
    return FE_OK;
}

}  // extern "C"
