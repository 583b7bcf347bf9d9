// Driver for the host-code sanitizer check of libmpsparse (test infrastructure).
//
// Built from the library's sources with the host half of every translation unit under
// AddressSanitizer and UndefinedBehaviorSanitizer (the device code is compiled as
// usual), it calls every C-ABI entry point on small matrices -- plan kinds, the SpMV
// variants, the argument and workspace checks, transpose and COO -> CSR, the DD and
// K-component solvers, refinement, the batched layer, the network and the
// allocation-free SpMV -- and checks their status codes and a few exact identities
// (the plan-free SpMV equals the explicit canonical plan's bit for bit; CG on an SPD
// tridiagonal system converges).  Every buffer is sized from the header's rules, so
// all device accesses stay in bounds.  Prints "ok" when every check held; the
// sanitizers abort or print their own reports otherwise.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "mpsparse.h"

static int g_fail = 0;

#define EXPECT(call, want)                                                                                    \
    do {                                                                                                      \
        const mp_status s_ = (call);                                                                          \
        if (s_ != (want)) {                                                                                   \
            std::fprintf(stderr, "line %d: %s returned %d, expected %d (%s)\n", __LINE__, #call, (int)s_,     \
                         (int)(want), mp_last_error());                                                       \
            g_fail = 1;                                                                                       \
        }                                                                                                     \
    } while (0)
#define OK(call) EXPECT(call, MP_OK)

#define CHECK(cond)                                                                    \
    do {                                                                               \
        if (!(cond)) {                                                                 \
            std::fprintf(stderr, "line %d: check failed: %s\n", __LINE__, #cond);     \
            g_fail = 1;                                                                \
        }                                                                              \
    } while (0)

static void hip_or_die(hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        std::fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
        std::exit(2);
    }
}

template <typename T>
static T *dev_alloc(size_t n)
{
    void *p = nullptr;
    hip_or_die(hipMalloc(&p, sizeof(T) * (n ? n : 1)), "hipMalloc");
    return static_cast<T *>(p);
}

template <typename T>
static T *dev_copy(const std::vector<T> &h)
{
    T *d = dev_alloc<T>(h.size());
    if (!h.empty()) hip_or_die(hipMemcpy(d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice), "hipMemcpy");
    return d;
}

template <typename T>
static std::vector<T> host_copy(const T *d, size_t n)
{
    std::vector<T> h(n);
    hip_or_die(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (n) hip_or_die(hipMemcpy(h.data(), d, sizeof(T) * n, hipMemcpyDeviceToHost), "hipMemcpy");
    return h;
}

// small deterministic generator (xorshift64*), uniform in (-1, 1)
struct Rng {
    uint64_t s;
    explicit Rng(uint64_t seed) : s(seed * 2654435761u + 1) {}
    double uni()
    {
        s ^= s >> 12;
        s ^= s << 25;
        s ^= s >> 27;
        const uint64_t v = s * 2685821657736338717ull;
        return ((double)(v >> 11) / 9007199254740992.0) * 2.0 - 1.0;
    }
};

// K-component planar values: lead from f(i), each further component 2^-53 u times the last
static std::vector<double> mp_values(size_t count, int K, Rng &rng, double (*lead)(size_t, Rng &))
{
    std::vector<double> v((size_t)K * count);
    for (size_t i = 0; i < count; ++i) {
        double c = lead(i, rng);
        v[i] = c;
        for (int k = 1; k < K; ++k) {
            c = c * std::ldexp(rng.uni(), -53);
            v[(size_t)k * count + i] = c;
        }
    }
    return v;
}

static double lead_uniform(size_t, Rng &rng) { return rng.uni(); }

struct HostCsr {
    int32_t n = 0, m = 0;
    std::vector<int32_t> rp, ci;
};

struct DevCsr {
    mp_csr c{};
    int32_t *rp = nullptr, *ci = nullptr;
    explicit DevCsr(const HostCsr &h)
    {
        rp = dev_copy(h.rp);
        ci = dev_copy(h.ci);
        c.n_rows = h.n;
        c.n_cols = h.m;
        c.nnz = (int64_t)h.ci.size();
        c.row_ptr = rp;
        c.col_idx = ci;
    }
    ~DevCsr()
    {
        (void)hipFree(rp);
        (void)hipFree(ci);
    }
};

// block-diagonal tridiagonal systems (SPD, symmetric pattern): diagonal 4, off-diagonal -1
static HostCsr tridiag_blocks(const std::vector<int32_t> &sizes, std::vector<double> &lead)
{
    HostCsr h;
    h.rp.push_back(0);
    int32_t off = 0;
    for (int32_t sz : sizes) {
        for (int32_t i = 0; i < sz; ++i) {
            if (i > 0) {
                h.ci.push_back(off + i - 1);
                lead.push_back(-1.0);
            }
            h.ci.push_back(off + i);
            lead.push_back(4.0 + 0.25 * (i % 3));
            if (i + 1 < sz) {
                h.ci.push_back(off + i + 1);
                lead.push_back(-1.0);
            }
            h.rp.push_back((int32_t)h.ci.size());
        }
        off += sz;
    }
    h.n = h.m = off;
    return h;
}

// ragged rows: empty rows, short rows and a few long ones (up to 1500 elements), sorted columns
static HostCsr ragged(int32_t n)
{
    HostCsr h;
    h.n = h.m = n;
    h.rp.push_back(0);
    for (int32_t i = 0; i < n; ++i) {
        int32_t len = (i % 97 == 0) ? 1500 - (i % 5) * 200 : (i % 11 == 0 ? 0 : 1 + (i * 7) % 40);
        if (len > n) len = n;
        std::vector<int32_t> cols;
        for (int32_t k = 0; k < len; ++k) cols.push_back((int32_t)(((int64_t)i * 13 + (int64_t)k * 3) % n));
        std::sort(cols.begin(), cols.end());
        cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
        h.ci.insert(h.ci.end(), cols.begin(), cols.end());
        h.rp.push_back((int32_t)h.ci.size());
    }
    return h;
}

typedef mp_status (*spmv_real_fn)(const mp_csr *, const double *, const double *, double *, const mp_plan *, void *,
                                  size_t, void *);
typedef mp_status (*spmv_cplx_fn)(const mp_csr *, const double *, const double *, const double *, const double *,
                                  double *, double *, const mp_plan *, void *, size_t, void *);

static spmv_real_fn real_fn(int K, bool dm)
{
    if (dm) return K == 2 ? mpspmv_csr_dd_d : K == 3 ? mpspmv_csr_td_d : mpspmv_csr_qd_d;
    return K == 2 ? mpspmv_csr_dd : K == 3 ? mpspmv_csr_td : mpspmv_csr_qd;
}

static spmv_cplx_fn cplx_fn(int K, bool dm)
{
    if (dm) return K == 2 ? mpspmv_csr_dd_d_complex : K == 3 ? mpspmv_csr_td_d_complex : mpspmv_csr_qd_d_complex;
    return K == 2 ? mpspmv_csr_dd_complex : K == 3 ? mpspmv_csr_td_complex : mpspmv_csr_qd_complex;
}

// canonical lane widths: log2 of the largest power of two <= min(len, 64)
static std::vector<uint8_t> canonical_log2w(const HostCsr &h)
{
    std::vector<uint8_t> lw((size_t)h.n, 0);
    for (int32_t i = 0; i < h.n; ++i) {
        const int32_t len = h.rp[i + 1] - h.rp[i];
        int w = 0;
        while (w < 6 && (2 << w) <= len) ++w;
        lw[i] = (uint8_t)w;
    }
    return lw;
}

static void spmv_section()
{
    const HostCsr H = ragged(2000);
    DevCsr A(H);
    const size_t nnz = H.ci.size(), n = (size_t)H.n;
    Rng rng(7);
    const std::vector<double> are = mp_values(nnz, 4, rng, lead_uniform), aim = mp_values(nnz, 4, rng, lead_uniform);
    const std::vector<double> xre = mp_values(n, 4, rng, lead_uniform), xim = mp_values(n, 4, rng, lead_uniform);
    OK(mp_csr_validate(&A.c, nullptr));
    const mp_plan_opts opts_list[] = {{0, 6, 0, 0}, {2, 6, 512, 0}, {1, 8, 256, 0}, {0, 10, 0, 0},
                                      {2, 6, 512, 1}, {1, 6, 256, 2}, {3, 5, 1024, 0}};
    for (int K = 2; K <= 4; ++K) {
        for (int cplx = 0; cplx <= 1; ++cplx) {
            // K-component operands: the leading K components of the 4-component draws
            std::vector<double> a_re(are.begin(), are.begin() + (long)(K * nnz));
            std::vector<double> a_im(aim.begin(), aim.begin() + (long)(K * nnz));
            std::vector<double> x_re(xre.begin(), xre.begin() + (long)(K * n));
            std::vector<double> x_im(xim.begin(), xim.begin() + (long)(K * n));
            double *dar = dev_copy(a_re), *dai = dev_copy(a_im), *dxr = dev_copy(x_re), *dxi = dev_copy(x_im);
            double *dyr = dev_alloc<double>((size_t)K * n), *dyi = dev_alloc<double>((size_t)K * n);
            double *a64r = dev_copy(std::vector<double>(are.begin(), are.begin() + (long)nnz));
            double *a64i = dev_copy(std::vector<double>(aim.begin(), aim.begin() + (long)nnz));
            for (const mp_plan_opts &o : opts_list) {
                mp_plan *plan = nullptr;
                const mp_status st = mp_plan_create(&A.c, K, cplx, &o, nullptr, &plan);
                if (st == MP_ERR_UNSUPPORTED) continue;   // tile size beyond this variant's LDS budget
                OK(st);
                if (!plan) continue;
                int32_t nr = 0, nt = 0, tn = 0, nc = 0, ic = 0;
                OK(mp_plan_info(plan, &nr, &nt, &tn, &nc, &ic));
                CHECK(nr == H.n && nc == K && ic == cplx);
                std::vector<uint8_t> lw(n);
                OK(mp_plan_row_log2w(plan, lw.data()));
                size_t wb = 0;
                OK(mpspmv_workspace_bytes(plan, &wb));
                void *ws = wb ? dev_alloc<char>(wb) : nullptr;
                for (int dm = 0; dm <= 1; ++dm) {
                    const double *ar = dm ? a64r : dar, *ai = dm ? a64i : dai;
                    if (cplx)
                        OK(cplx_fn(K, dm)(&A.c, ar, ai, dxr, dxi, dyr, dyi, plan, ws, wb, nullptr));
                    else
                        OK(real_fn(K, dm)(&A.c, ar, dxr, dyr, plan, ws, wb, nullptr));
                }
                (void)hipFree(ws);
                OK(mp_plan_destroy(plan));
            }
            // the plan-free kernel and an explicit plan of the canonical order agree bit for bit
            const std::vector<uint8_t> lw = canonical_log2w(H);
            mp_plan *ep = nullptr;
            OK(mp_plan_create_explicit(&A.c, K, cplx, lw.data(), 0, nullptr, &ep));
            size_t wb = 0;
            OK(mpspmv_workspace_bytes(ep, &wb));
            void *ws = wb ? dev_alloc<char>(wb) : nullptr;
            double *dzr = dev_alloc<double>((size_t)K * n), *dzi = dev_alloc<double>((size_t)K * n);
            if (cplx) {
                OK(cplx_fn(K, false)(&A.c, dar, dai, dxr, dxi, dyr, dyi, nullptr, nullptr, 0, nullptr));
                OK(cplx_fn(K, false)(&A.c, dar, dai, dxr, dxi, dzr, dzi, ep, ws, wb, nullptr));
                CHECK(host_copy(dyi, (size_t)K * n) == host_copy(dzi, (size_t)K * n));
            } else {
                OK(real_fn(K, false)(&A.c, dar, dxr, dyr, nullptr, nullptr, 0, nullptr));
                OK(real_fn(K, false)(&A.c, dar, dxr, dzr, ep, ws, wb, nullptr));
            }
            CHECK(host_copy(dyr, (size_t)K * n) == host_copy(dzr, (size_t)K * n));
            OK(mp_plan_destroy(ep));
            (void)hipFree(ws);
            (void)hipFree(dzr);
            (void)hipFree(dzi);
            (void)hipFree(dar);
            (void)hipFree(dai);
            (void)hipFree(dxr);
            (void)hipFree(dxi);
            (void)hipFree(dyr);
            (void)hipFree(dyi);
            (void)hipFree(a64r);
            (void)hipFree(a64i);
        }
    }

    // autotuner (one repetition per trial) and the argument / workspace checks of a DD call
    double *da = dev_copy(std::vector<double>(are.begin(), are.begin() + (long)(2 * nnz)));
    double *dx = dev_copy(std::vector<double>(xre.begin(), xre.begin() + (long)(2 * n)));
    double *dy = dev_alloc<double>(2 * n);
    mp_plan *tp = nullptr;
    mp_plan_opts chosen{};
    OK(mp_plan_autotune(&A.c, 2, 0, da, nullptr, dx, nullptr, dy, nullptr, 1, nullptr, &tp, &chosen));
    size_t wb = 0;
    OK(mpspmv_workspace_bytes(tp, &wb));
    CHECK(wb > 0);
    char *ws = dev_alloc<char>(wb + 256);
    OK(mpspmv_csr_dd(&A.c, da, dx, dy, tp, ws, wb, nullptr));
    OK(mpspmv_csr_dd_noalloc(&A.c, da, dx, dy, tp, nullptr));
    OK(mpspmv_csr_dd_noalloc(&A.c, da, dx, dy, nullptr, nullptr));
    EXPECT(mpspmv_csr_dd(&A.c, da, dx, nullptr, tp, ws, wb, nullptr), MP_ERR_INVALID_ARG);
    CHECK(std::strlen(mp_last_error()) > 0);
    EXPECT(mpspmv_csr_dd(&A.c, da, dx, dx, tp, ws, wb, nullptr), MP_ERR_ALIAS);
    EXPECT(mpspmv_csr_dd(&A.c, da, dx, dy, tp, ws, wb - 1, nullptr), MP_ERR_NO_MEMORY);
    EXPECT(mpspmv_csr_dd(&A.c, da, dx, dy, tp, nullptr, 0, nullptr), MP_ERR_INVALID_ARG);
    EXPECT(mpspmv_csr_dd(&A.c, da, dx, dy, tp, ws + 8, wb, nullptr), MP_ERR_INVALID_ARG);
    EXPECT(mpspmv_csr_td(&A.c, da, dx, dy, tp, ws, wb, nullptr), MP_ERR_INVALID_ARG);   // a DD plan
    EXPECT(mpspmv_csr_dd(nullptr, da, dx, dy, tp, ws, wb, nullptr), MP_ERR_INVALID_ARG);
    mp_plan *bad = nullptr;
    const mp_plan_opts bad_opts[] = {{13, 6, 0, 0}, {0, 11, 0, 0}, {0, 6, 300, 0}, {0, 6, 0, 3}, {-1, 6, 0, 0}};
    for (const mp_plan_opts &o : bad_opts) EXPECT(mp_plan_create(&A.c, 2, 0, &o, nullptr, &bad), MP_ERR_INVALID_ARG);
    EXPECT(mp_plan_create(&A.c, 5, 0, nullptr, nullptr, &bad), MP_ERR_INVALID_ARG);
    // a plan of another matrix
    std::vector<double> tl;
    const HostCsr T = tridiag_blocks({2000}, tl);
    DevCsr B(T);
    EXPECT(mpspmv_csr_dd(&B.c, da, dx, dy, tp, ws, wb, nullptr), MP_ERR_INVALID_ARG);
    OK(mp_plan_destroy(tp));
    OK(mp_plan_destroy(nullptr));
    // a malformed CSR: decreasing row pointers
    HostCsr M = H;
    M.rp[5] = M.rp[6] + 1;
    DevCsr Bad(M);
    EXPECT(mp_csr_validate(&Bad.c, nullptr), MP_ERR_INVALID_ARG);
    EXPECT(mp_csr_validate(nullptr, nullptr), MP_ERR_INVALID_ARG);
    // z = x - y, in place and with a partial overlap (refused)
    OK(mpvec_dd_sub((int64_t)n, dx, dy, dy, nullptr));
    EXPECT(mpvec_dd_sub((int64_t)n - 1, dx, dy, dx + 1, nullptr), MP_ERR_ALIAS);
    (void)hipFree(ws);
    (void)hipFree(da);
    (void)hipFree(dx);
    (void)hipFree(dy);
}

static void layout_section()
{
    const HostCsr H = ragged(700);
    DevCsr A(H);
    const size_t nnz = H.ci.size(), n = (size_t)H.n;
    Rng rng(11);
    for (int K = 1; K <= 4; ++K) {
        for (int cplx = 0; cplx <= 1; ++cplx) {
            double *ar = dev_copy(mp_values(nnz, K, rng, lead_uniform));
            double *ai = cplx ? dev_copy(mp_values(nnz, K, rng, lead_uniform)) : nullptr;
            int32_t *rpt = dev_alloc<int32_t>(n + 1), *cit = dev_alloc<int32_t>(nnz);
            double *atr = dev_alloc<double>((size_t)K * nnz), *ati = cplx ? dev_alloc<double>((size_t)K * nnz) : nullptr;
            OK(mp_csr_transpose(&A.c, K, ar, ai, rpt, cit, atr, ati, nullptr));
            EXPECT(mp_csr_transpose(&A.c, K, ar, ai, rpt, cit, ar, ati, nullptr), MP_ERR_ALIAS);
            // COO of the same elements in reverse order, plus duplicates of the first 50
            std::vector<int32_t> row, col;
            for (int32_t i = 0; i < H.n; ++i)
                for (int32_t k = H.rp[i]; k < H.rp[i + 1]; ++k) {
                    row.push_back(i);
                    col.push_back(H.ci[k]);
                }
            std::vector<int32_t> rrow(row.rbegin(), row.rend()), rcol(col.rbegin(), col.rend());
            for (int k = 0; k < 50; ++k) {
                rrow.push_back(row[(size_t)k]);
                rcol.push_back(col[(size_t)k]);
            }
            const size_t cn = rrow.size();
            int32_t *dr = dev_copy(rrow), *dc = dev_copy(rcol);
            double *vr = dev_copy(mp_values(cn, K, rng, lead_uniform));
            double *vi = cplx ? dev_copy(mp_values(cn, K, rng, lead_uniform)) : nullptr;
            int32_t *orp = dev_alloc<int32_t>(n + 1), *oci = dev_alloc<int32_t>(cn);
            double *oar = dev_alloc<double>((size_t)K * cn), *oai = cplx ? dev_alloc<double>((size_t)K * cn) : nullptr;
            OK(mp_coo_to_csr(H.n, H.m, (int64_t)cn, dr, dc, K, vr, vi, orp, oci, oar, oai, nullptr));
            const std::vector<int32_t> hrp = host_copy(orp, n + 1);
            CHECK(hrp[0] == 0 && hrp[n] == (int32_t)cn);
            // a coordinate outside the matrix: refused, nothing written
            std::vector<int32_t> brow = rrow;
            brow[3] = H.n;
            int32_t *dbr = dev_copy(brow);
            EXPECT(mp_coo_to_csr(H.n, H.m, (int64_t)cn, dbr, dc, K, vr, vi, orp, oci, oar, oai, nullptr),
                   MP_ERR_INVALID_ARG);
            EXPECT(mp_coo_to_csr(H.n, H.m, (int64_t)cn, dr, dc, 5, vr, vi, orp, oci, oar, oai, nullptr),
                   MP_ERR_INVALID_ARG);
            for (void *p : {(void *)ar, (void *)ai, (void *)rpt, (void *)cit, (void *)atr, (void *)ati, (void *)dr,
                            (void *)dc, (void *)vr, (void *)vi, (void *)orp, (void *)oci, (void *)oar, (void *)oai,
                            (void *)dbr})
                if (p) (void)hipFree(p);
        }
    }
}

static mp_solve_opts solve_opts(double rtol, int max_iter)
{
    mp_solve_opts o{};
    o.precond = MP_PRECOND_JACOBI;
    o.max_iter = max_iter;
    o.rtol = rtol;
    o.check_every = 16;
    o.inner = MP_INNER_FP64;
    o.inner_rtol = 1e-8;
    o.inner_max_iter = 0;
    o.max_outer = 40;
    return o;
}

static void solver_section()
{
    std::vector<double> lead;
    const HostCsr H = tridiag_blocks({9000}, lead);   // three dot chunks
    DevCsr A(H);
    const size_t nnz = H.ci.size(), n = (size_t)H.n;
    Rng rng(5);
    std::vector<double> a4((size_t)4 * nnz, 0.0);
    for (size_t k = 0; k < nnz; ++k) a4[k] = lead[k];   // exact leads, zero tails
    const std::vector<double> b4 = mp_values(n, 4, rng, lead_uniform);
    mp_solve_info info{};

    // DD solvers
    double *a = dev_copy(std::vector<double>(a4.begin(), a4.begin() + (long)(2 * nnz)));
    double *b = dev_copy(std::vector<double>(b4.begin(), b4.begin() + (long)(2 * n)));
    double *x = dev_alloc<double>(2 * n);
    int32_t *rpt = dev_alloc<int32_t>(n + 1), *cit = dev_alloc<int32_t>(nnz);
    double *at = dev_alloc<double>(2 * nnz);
    OK(mp_csr_transpose(&A.c, 2, a, nullptr, rpt, cit, at, nullptr, nullptr));
    mp_csr At = A.c;
    At.row_ptr = rpt;
    At.col_idx = cit;
    mp_plan *plan = nullptr, *plan_t = nullptr;
    const mp_plan_opts po{1, 6, 0, 0};
    OK(mp_plan_create(&A.c, 2, 0, &po, nullptr, &plan));
    OK(mp_plan_create(&At, 2, 0, &po, nullptr, &plan_t));
    for (int inner = 0; inner <= 1; ++inner) {
        mp_solve_opts o = solve_opts(1e-26, 20000);
        o.inner = inner ? MP_INNER_FP32 : MP_INNER_FP64;
        o.inner_rtol = inner ? 1e-5 : 1e-8;
        size_t wb = 0;
        OK(mpkrylov_workspace_bytes(&A.c, &o, &wb));
        void *ws = dev_alloc<char>(wb);
        const size_t zb = 2 * n * sizeof(double);
        hip_or_die(hipMemset(x, 0, zb), "hipMemset");
        OK(mpkrylov_cg(&A.c, a, b, x, &o, plan, ws, wb, &info, nullptr));
        CHECK(info.status == MP_OK && info.relres <= 1e-26 && info.iters > 0);
        hip_or_die(hipMemset(x, 0, zb), "hipMemset");
        OK(mpkrylov_bicgstab(&A.c, a, b, x, &o, plan, ws, wb, &info, nullptr));
        hip_or_die(hipMemset(x, 0, zb), "hipMemset");
        OK(mpkrylov_cgs(&A.c, a, b, x, &o, plan, ws, wb, &info, nullptr));
        hip_or_die(hipMemset(x, 0, zb), "hipMemset");
        OK(mpkrylov_gpbicg(&A.c, a, b, x, &o, plan, ws, wb, &info, nullptr));
        hip_or_die(hipMemset(x, 0, zb), "hipMemset");
        OK(mpkrylov_bicg(&A.c, a, &At, at, b, x, &o, plan, plan_t, ws, wb, &info, nullptr));
        hip_or_die(hipMemset(x, 0, zb), "hipMemset");
        OK(mpkrylov_ir(&A.c, a, b, x, &o, plan, ws, wb, &info, nullptr));
        CHECK(info.outer_iters > 0);
        hip_or_die(hipMemset(x, 0, zb), "hipMemset");
        mp_solve_opts lim = o;
        lim.max_iter = 3;
        EXPECT(mpkrylov_cg(&A.c, a, b, x, &lim, plan, ws, wb, &info, nullptr), MP_ERR_NOT_CONVERGED);
        CHECK(info.status == MP_ERR_NOT_CONVERGED && info.iters > 0 && info.iters <= 3);
        // the refinement needs all of wb (binary32: a copy of hi(A) besides the vectors), CG less
        EXPECT(mpkrylov_ir(&A.c, a, b, x, &o, plan, ws, wb - 1, &info, nullptr), MP_ERR_NO_MEMORY);
        EXPECT(mpkrylov_cg(&A.c, a, b, x, &o, plan, ws, 1024, &info, nullptr), MP_ERR_NO_MEMORY);
        EXPECT(mpkrylov_cg(&A.c, a, b, b, &o, plan, ws, wb, &info, nullptr), MP_ERR_ALIAS);
        (void)hipFree(ws);
    }
    OK(mp_plan_destroy(plan));
    OK(mp_plan_destroy(plan_t));

    // K-component solvers
    for (int K = 3; K <= 4; ++K) {
        double *ak = dev_copy(std::vector<double>(a4.begin(), a4.begin() + (long)((size_t)K * nnz)));
        double *atk = dev_alloc<double>((size_t)K * nnz);
        OK(mp_csr_transpose(&A.c, K, ak, nullptr, rpt, cit, atk, nullptr, nullptr));
        double *bk = dev_copy(std::vector<double>(b4.begin(), b4.begin() + (long)((size_t)K * n)));
        double *xk = dev_alloc<double>((size_t)K * n);
        mp_plan *pk = nullptr, *pkt = nullptr;
        OK(mp_plan_create(&A.c, K, 0, &po, nullptr, &pk));
        OK(mp_plan_create(&At, K, 0, &po, nullptr, &pkt));
        size_t wb = 0;
        OK(mpkrylov_mp_workspace_bytes(&A.c, K, &wb));
        void *ws = dev_alloc<char>(wb);
        const mp_solve_opts o = solve_opts(K == 3 ? 1e-40 : 1e-55, 20000);
        const size_t zb = (size_t)K * n * sizeof(double);
        typedef mp_status (*solver)(const mp_csr *, const double *, const double *, double *, const mp_solve_opts *,
                                    const mp_plan *, void *, size_t, mp_solve_info *, void *);
        const solver list[] = {K == 3 ? mpkrylov_cg_td : mpkrylov_cg_qd,
                               K == 3 ? mpkrylov_bicgstab_td : mpkrylov_bicgstab_qd,
                               K == 3 ? mpkrylov_cgs_td : mpkrylov_cgs_qd,
                               K == 3 ? mpkrylov_gpbicg_td : mpkrylov_gpbicg_qd};
        for (solver f : list) {
            hip_or_die(hipMemset(xk, 0, zb), "hipMemset");
            OK(f(&A.c, ak, bk, xk, &o, pk, ws, wb, &info, nullptr));
        }
        hip_or_die(hipMemset(xk, 0, zb), "hipMemset");
        OK((K == 3 ? mpkrylov_bicg_td : mpkrylov_bicg_qd)(&A.c, ak, &At, atk, bk, xk, &o, pk, pkt, ws, wb, &info,
                                                           nullptr));
        OK(mp_plan_destroy(pk));
        OK(mp_plan_destroy(pkt));
        for (void *p : {(void *)ak, (void *)atk, (void *)bk, (void *)xk, ws}) (void)hipFree(p);
    }

    // the network: parameters, graph, forward, loss and gradients, Adam, learned refinement
    int32_t np = 0;
    OK(mp_mpnn_param_count(&np));
    CHECK(np > 0);
    mp_mpnn *net = nullptr;
    EXPECT(mp_mpnn_create(32, &net), MP_ERR_UNSUPPORTED);
    OK(mp_mpnn_create(64, &net));
    std::vector<float> theta((size_t)np), grads((size_t)np);
    for (float &t : theta) t = (float)(0.02 * rng.uni());
    OK(mp_mpnn_set_params(net, theta.data()));
    mp_graph *g = nullptr;
    OK(mp_graph_create(&A.c, a, nullptr, &g));
    double *mv = dev_alloc<double>(nnz);
    OK(mp_mpnn_forward(net, g, mv, nullptr));
    const int npairs = 2;
    double *r = dev_copy(mp_values((size_t)npairs * n, 1, rng, lead_uniform));
    double *e = dev_copy(mp_values((size_t)npairs * n, 1, rng, lead_uniform));
    double loss[npairs] = {0, 0};
    OK(mp_mpnn_zero_grads(net, nullptr));
    OK(mp_mpnn_loss_grad(net, g, r, e, npairs, loss, nullptr));
    CHECK(std::isfinite(loss[0]) && std::isfinite(loss[1]));
    OK(mp_mpnn_adam_step(net, 1e-3f, 0.9f, 0.999f, 1e-8f, 0.5f, 1, nullptr));
    OK(mp_mpnn_get_params(net, theta.data()));
    OK(mp_mpnn_get_grads(net, grads.data()));
    mp_solve_opts lo = solve_opts(1e-26, 20000);
    lo.precond = MP_PRECOND_LEARNED;
    size_t wb = 0;
    OK(mpkrylov_workspace_bytes(&A.c, &lo, &wb));
    void *ws = dev_alloc<char>(wb);
    hip_or_die(hipMemset(x, 0, 2 * n * sizeof(double)), "hipMemset");
    OK(mpkrylov_ir_learned(&A.c, a, mv, b, x, &lo, nullptr, ws, wb, &info, nullptr));
    EXPECT(mpkrylov_ir_learned(&A.c, a, x, b, x, &lo, nullptr, ws, wb, &info, nullptr), MP_ERR_ALIAS);
    OK(mp_graph_destroy(g));
    OK(mp_mpnn_destroy(net));
    for (void *p : {(void *)a, (void *)b, (void *)x, (void *)rpt, (void *)cit, (void *)at, (void *)mv, (void *)r,
                    (void *)e, ws})
        (void)hipFree(p);
}

static void batched_section()
{
    std::vector<double> lead;
    const std::vector<int32_t> sizes = {100, 5000, 300};
    const HostCsr H = tridiag_blocks(sizes, lead);
    DevCsr A(H);
    const size_t nnz = H.ci.size(), N = (size_t)H.n;
    const int32_t R = 4;
    std::vector<int32_t> sp = {0};
    for (int32_t s : sizes) sp.push_back(sp.back() + s);
    std::vector<double> a2(2 * nnz, 0.0);
    for (size_t k = 0; k < nnz; ++k) a2[k] = lead[k];
    Rng rng(9);
    double *a = dev_copy(a2);
    double *B = dev_copy(mp_values(N * R, 2, rng, lead_uniform));
    double *X = dev_alloc<double>(2 * N * R), *Y = dev_alloc<double>(2 * N * R);
    hip_or_die(hipMemset(X, 0, 2 * N * R * sizeof(double)), "hipMemset");
    mp_batch_plan *bp = nullptr;
    EXPECT(mp_batch_plan_create(&A.c, sp.data(), 3, R, 3, nullptr, &bp), MP_ERR_INVALID_ARG);
    OK(mp_batch_plan_create(&A.c, sp.data(), 3, R, 1, nullptr, &bp));
    int32_t tpr = 0, rows = 0, order = 0;
    OK(mp_batch_plan_autotune(bp, &A.c, a, B, Y, 1, nullptr, &tpr));
    OK(mp_batch_plan_schedule(bp, &tpr, &rows, &order));
    CHECK(tpr >= 1 && tpr <= R && rows > 0);
    EXPECT(mp_batch_plan_set_schedule(bp, 3, 1, 0), MP_ERR_INVALID_ARG);
    OK(mp_batch_plan_set_schedule(bp, 2, 2, 1));
    OK(mpspmm_csr_dd_batched(&A.c, a, B, Y, R, bp, nullptr));
    OK(mpspmm_csr_dd_batched(&A.c, a, B, Y, R, nullptr, nullptr));
    size_t wb = 0;
    OK(mpkrylov_batched_workspace_bytes(bp, &wb));
    void *ws = dev_alloc<char>(wb);
    std::vector<mp_solve_info> infos((size_t)3 * R);
    const mp_solve_opts o = solve_opts(1e-26, 20000);
    for (int graph = 0; graph <= 1; ++graph) {
        hip_or_die(hipMemset(X, 0, 2 * N * R * sizeof(double)), "hipMemset");
        OK(mpkrylov_cg_batched(&A.c, a, B, X, R, &o, bp, graph, ws, wb, infos.data(), nullptr));
        for (const mp_solve_info &i : infos) CHECK(i.status == MP_OK && i.relres <= 1e-26);
    }
    EXPECT(mpkrylov_cg_batched(&A.c, a, B, X, R, &o, bp, 0, ws, wb - 1, infos.data(), nullptr), MP_ERR_NO_MEMORY);
    OK(mp_batch_plan_destroy(bp));
    for (void *p : {(void *)a, (void *)B, (void *)X, (void *)Y, ws}) (void)hipFree(p);
}

int main(int argc, char **argv)
{
    std::printf("library %s\n", mp_version());
    if (argc > 1 && std::strcmp(argv[1], "--version") == 0) return 0;
    double rate = 0.0;
    EXPECT(mp_measure_rate(1, &rate, nullptr), MP_ERR_INVALID_ARG);
    std::printf("spmv\n");
    std::fflush(stdout);
    spmv_section();
    std::printf("layout\n");
    std::fflush(stdout);
    layout_section();
    std::printf("solvers\n");
    std::fflush(stdout);
    solver_section();
    std::printf("batched\n");
    std::fflush(stdout);
    batched_section();
    hip_or_die(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (g_fail) {
        std::printf("FAILED\n");
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
