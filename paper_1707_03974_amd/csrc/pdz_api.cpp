// Host runtime of the pdz C ABI: validation, problem set-up, dispatch.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pdz_internal.h"

namespace pdz {

namespace {
thread_local std::string g_last_error;
std::mutex g_ctx_mutex;
DeviceCtx g_ctx[64];
}  // namespace

pdz_status fail(pdz_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

pdz_status ok() { return PDZ_OK; }

pdz_status hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? PDZ_ENOMEM : PDZ_EHIP;
}

pdz_status device_ctx(DeviceCtx** out) {
    int dev = 0;
    PDZ_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(PDZ_ERANGE, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_ctx_mutex);
    DeviceCtx& c = g_ctx[dev];
    if (c.device < 0) {
        hipDeviceProp_t prop;
        PDZ_HIP(hipGetDeviceProperties(&prop, dev));
        PDZ_HIP(hipMalloc(&c.err, 256));
        PDZ_HIP(hipMemset(c.err, 0, 256));
        std::vector<uint32_t> C;
        binomial_table(C);
        PDZ_HIP(hipMalloc(&c.binom, C.size() * sizeof(uint32_t)));
        PDZ_HIP(hipMemcpy(c.binom, C.data(), C.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
        pdz_status hs = hv_prepare();
        if (hs == PDZ_OK) hs = batch_prepare();
        if (hs == PDZ_OK) hs = kspace_prepare();
        if (hs == PDZ_OK) hs = parity_prepare();
        if (hs != PDZ_OK) return hs;
        c.cu_count = prop.multiProcessorCount;
        c.lds_per_block = prop.sharedMemPerBlock;
        c.device = dev;
    }
    *out = &c;
    return ok();
}

// Binomial coefficients by Pascal's rule C_i^m = C_{i-1}^m + C_{i-1}^{m-1}
// (Sec. III), with C_i^0 = 1 and C_i^m = 0 for m > i.
void binomial_table(std::vector<uint32_t>& C) {
    C.assign(kBinomStride * kBinomStride, 0u);
    for (int i = 0; i <= kMaxSites; ++i) {
        C[i * kBinomStride + 0] = 1u;
        for (int m = 1; m <= i; ++m)
            C[i * kBinomStride + m] = C[(i - 1) * kBinomStride + m] + C[(i - 1) * kBinomStride + m - 1];
    }
}

uint64_t binom(int n, int k) {
    if (k < 0 || k > n) return 0;
    uint64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
    return r;
}

pdz_status launch_hv_any(const pdz_problem_s* p, pdz_dtype dt, const void* x, void* y, hipStream_t s,
                         const int* skip, unsigned passes, const HvSplit* split, uint64_t pitch) {
    if ((p->ks || p->par) && pitch != 0) return fail(PDZ_EINVAL, "a symmetry-sector H.v takes unpadded vectors");
    if (p->ks) {
        if (split || passes != (kPassDown | kPassUp))
            return fail(PDZ_EINVAL, "a momentum-space H.v has no separate passes");
        return launch_hvk(p, dt, x, y, s, skip);
    }
    if (p->par) return launch_hvp_split(p, dt, x, y, s, skip, passes, split);
    return launch_hv(p, dt, x, y, s, skip, passes, split, pitch);
}

}  // namespace pdz

using namespace pdz;

static void free_tables(SectorTables& t) {
    if (t.states) (void)hipFree(t.states);
    if (t.count) (void)hipFree(t.count);
    if (t.ell) (void)hipFree(t.ell);
    if (t.ell16) (void)hipFree(t.ell16);
    free_down_schedule(&t.sched);
    t.ell16 = nullptr;
    t.states = nullptr;
    t.count = nullptr;
    t.ell = nullptr;
}

static void destroy_problem(pdz_problem_s* p) {
    if (!p) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    free_tables(p->up);
    if (!p->same_sector) free_tables(p->dn);
    if (p->d_binom) (void)hipFree(p->d_binom);
    if (p->d_bonds) (void)hipFree(p->d_bonds);
    if (p->d_coef64) (void)hipFree(p->d_coef64);
    if (p->d_coef32) (void)hipFree(p->d_coef32);
    kspace_free(p->ks);
    parity_free(p->par);
    (void)hipSetDevice(prev);
    delete p;
}

extern "C" {

const char* pdz_last_error(void) { return g_last_error.c_str(); }

int32_t pdz_version(void) { return 100; }

pdz_status pdz_problem_create(int32_t n_sites, const pdz_bond* bonds, int32_t n_bonds, double U, int32_t n_up,
                              int32_t n_dn, pdz_problem* out) {
    g_last_error.clear();
    if (!out) return fail(PDZ_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_sites < 1 || n_sites > kMaxSites) return fail(PDZ_ERANGE, "n_sites must be in [1, 32]");
    if (n_bonds < 0) return fail(PDZ_EINVAL, "n_bonds < 0");
    if (n_bonds > 0 && !bonds) return fail(PDZ_EINVAL, "bonds is NULL");
    if (n_up < 0 || n_up > n_sites || n_dn < 0 || n_dn > n_sites)
        return fail(PDZ_EINVAL, "n_up and n_dn must be in [0, n_sites]");
    if (!std::isfinite(U)) return fail(PDZ_EINVAL, "U is not finite");
    for (int b = 0; b < n_bonds; ++b) {
        const pdz_bond& bd = bonds[b];
        if (bd.i < 0 || bd.i >= n_sites || bd.j < 0 || bd.j >= n_sites)
            return fail(PDZ_EINVAL, "bond " + std::to_string(b) + " has an endpoint outside [0, n_sites)");
        if (bd.i == bd.j) return fail(PDZ_EINVAL, "bond " + std::to_string(b) + " joins a site to itself");
        if (!std::isfinite(bd.t)) return fail(PDZ_EINVAL, "bond " + std::to_string(b) + " has a non-finite t");
    }
    const uint64_t D_up = binom(n_sites, n_up), D_dn = binom(n_sites, n_dn);
    if (D_up > 0 && D_dn > (1ull << 62) / D_up) return fail(PDZ_ERANGE, "D >= 2^62");

    DeviceCtx* ctx = nullptr;
    pdz_status st = device_ctx(&ctx);
    if (st != PDZ_OK) return st;

    pdz_problem_s* p = new pdz_problem_s();
    p->device = ctx->device;
    p->N = n_sites;
    p->n_up = n_up;
    p->n_dn = n_dn;
    p->n_bonds = n_bonds;
    p->U = U;
    p->bonds.assign(bonds, bonds + n_bonds);
    p->D = D_up * D_dn;
    p->up.D = D_up;
    p->up.n = n_up;
    p->dn.D = D_dn;
    p->dn.n = n_dn;

    // Signed hop amplitudes: -t for an even number of passed operators, +t for odd.
    std::vector<BondDev> bd(n_bonds > 0 ? n_bonds : 1);
    auto coef_index = [&](double v) -> int {
        for (size_t k = 0; k < p->coef_host.size(); ++k)
            if (p->coef_host[k] == v) return (int)k;
        p->coef_host.push_back(v);
        return (int)p->coef_host.size() - 1;
    };
    // Kernel bond order: bonds inside the upper half of the sites first, then
    // bonds across the halves, then bonds inside the lower half (stable).
    // States that share their upper half sit next to each other in a sector,
    // so their first hop slots name the same bond and land at one common
    // offset.  The sum over bonds is unchanged.
    std::vector<int> order(n_bonds);
    {
        const int half = n_sites / 2;
        auto cls = [&](int b) {
            const int hi_i = bonds[b].i >= half, hi_j = bonds[b].j >= half;
            return hi_i && hi_j ? 0 : (hi_i || hi_j ? 1 : 2);
        };
        int k = 0;
        for (int c = 0; c < 3; ++c)
            for (int b = 0; b < n_bonds; ++b)
                if (cls(b) == c) order[k++] = b;
    }
    for (int k = 0; k < n_bonds; ++k) {
        const int b = order[k];
        const int i = bonds[b].i, j = bonds[b].j;
        const int lo = i < j ? i : j, hi = i < j ? j : i;
        bd[k].mask = (1u << i) | (1u << j);
        uint32_t between = 0;
        for (int s = lo + 1; s < hi; ++s) between |= 1u << s;
        bd[k].between = between;
        bd[k].coef_pos = coef_index(-bonds[b].t);
        bd[k].coef_neg = coef_index(bonds[b].t);
    }
    if (p->coef_host.empty()) p->coef_host.push_back(0.0);
    if ((int)p->coef_host.size() > kMaxCoef) {
        destroy_problem(p);
        return fail(PDZ_ERANGE, "more than 256 distinct hopping amplitudes");
    }

    hipStream_t s = nullptr;
    std::vector<uint32_t> C;
    binomial_table(C);
    auto cleanup = [&](pdz_status code) {
        destroy_problem(p);
        return code;
    };
#define CK(call)                                            \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return cleanup(hip_fail(e_, #call)); \
    } while (0)
    CK(hipMalloc(&p->d_binom, C.size() * sizeof(uint32_t)));
    CK(hipMemcpy(p->d_binom, C.data(), C.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    CK(hipMalloc(&p->d_bonds, bd.size() * sizeof(BondDev)));
    CK(hipMemcpy(p->d_bonds, bd.data(), bd.size() * sizeof(BondDev), hipMemcpyHostToDevice));
    std::vector<float> c32(p->coef_host.begin(), p->coef_host.end());
    CK(hipMalloc(&p->d_coef64, kMaxCoef * sizeof(double)));
    CK(hipMalloc(&p->d_coef32, kMaxCoef * sizeof(float)));
    CK(hipMemset(p->d_coef64, 0, kMaxCoef * sizeof(double)));
    CK(hipMemset(p->d_coef32, 0, kMaxCoef * sizeof(float)));
    CK(hipMemcpy(p->d_coef64, p->coef_host.data(), p->coef_host.size() * sizeof(double), hipMemcpyHostToDevice));
    CK(hipMemcpy(p->d_coef32, c32.data(), c32.size() * sizeof(float), hipMemcpyHostToDevice));
#undef CK

    // Hop tables when every sector rank fits the 24-bit target field.  PDZ_HV_ONTHEFLY=1 selects the
    // path that ranks every hop target inside the H.v kernel instead (same summation order).
    const char* fly_env = std::getenv("PDZ_HV_ONTHEFLY");
    const bool force_fly = fly_env && fly_env[0] == '1';
    const bool tables = !force_fly && D_up <= (uint64_t)kTargetMask + 1 && D_dn <= (uint64_t)kTargetMask + 1;
    const uint64_t hops_closed_up = (n_sites >= 2 && n_up >= 1 && n_up < n_sites)
                                        ? 2ull * n_bonds * binom(n_sites - 2, n_up - 1) : 0ull;
    const uint64_t hops_closed_dn = (n_sites >= 2 && n_dn >= 1 && n_dn < n_sites)
                                        ? 2ull * n_bonds * binom(n_sites - 2, n_dn - 1) : 0ull;
    if (tables) {
        p->hv_path = 0;
        st = build_sector_tables(p->d_binom, n_sites, n_up, p->d_bonds, n_bonds, &p->up, ctx->err, s);
        if (st != PDZ_OK) return cleanup(st);
        st = build_compact_table(&p->up, (int)p->coef_host.size(), s);
        if (st != PDZ_OK) return cleanup(st);
        if (n_dn == n_up) {
            p->dn = p->up;
            p->same_sector = true;
        } else {
            st = build_sector_tables(p->d_binom, n_sites, n_dn, p->d_bonds, n_bonds, &p->dn, ctx->err, s);
            if (st != PDZ_OK) return cleanup(st);
            st = build_compact_table(&p->dn, (int)p->coef_host.size(), s);
            if (st != PDZ_OK) return cleanup(st);
        }
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) return cleanup(hip_fail(e, "table build"));
        // down-pass gather schedule (shared with the up tables when both sectors are one)
        st = build_down_schedule(p->dn, p->coef_host, &p->dn.sched, s);
        if (st != PDZ_OK) return cleanup(st);
        if (p->same_sector) p->up.sched = p->dn.sched;
        uint32_t word = 0;
        e = hipMemcpy(&word, ctx->err, sizeof(word), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return cleanup(hip_fail(e, "table build error word"));
        if (word & kErrTable) return cleanup(fail(PDZ_EDEVICE, "hop table build produced an out-of-range target"));
        if (p->up.total_hops != hops_closed_up || p->dn.total_hops != hops_closed_dn)
            return cleanup(fail(PDZ_EDEVICE, "hop count disagrees with 2 * n_bonds * C(N-2, n-1)"));
    } else {
        p->hv_path = 1;
        p->up.total_hops = hops_closed_up;
        p->dn.total_hops = hops_closed_dn;
    }
    p->nnz = p->D + p->up.total_hops * D_dn + p->dn.total_hops * D_up;
    *out = p;
    return ok();
}

pdz_status pdz_problem_destroy(pdz_problem p) {
    g_last_error.clear();
    destroy_problem(p);
    return ok();
}

pdz_status pdz_problem_info(pdz_problem p, pdz_info* out) {
    g_last_error.clear();
    if (!p || !out) return fail(PDZ_EINVAL, "NULL argument");
    out->D = p->D;
    out->D_up = p->up.D;
    out->D_dn = p->dn.D;
    out->nnz = p->nnz;
    out->hops_up = p->up.total_hops;
    out->hops_dn = p->dn.total_hops;
    out->n_sites = p->N;
    out->n_up = p->n_up;
    out->n_dn = p->n_dn;
    out->n_bonds = p->n_bonds;
    out->max_hops_up = p->up.max_hops;
    out->max_hops_dn = p->dn.max_hops;
    out->device = p->device;
    out->hv_path = p->hv_path;
    return ok();
}

pdz_status pdz_rank(int32_t n_sites, int32_t n, const uint32_t* bits, uint64_t count, uint32_t* ranks,
                    void* stream) {
    g_last_error.clear();
    if (n_sites < 1 || n_sites > kMaxSites) return fail(PDZ_ERANGE, "n_sites must be in [1, 32]");
    if (n < 0 || n > n_sites) return fail(PDZ_EINVAL, "n must be in [0, n_sites]");
    if (count > 0 && (!bits || !ranks)) return fail(PDZ_EINVAL, "NULL array");
    DeviceCtx* ctx = nullptr;
    pdz_status st = device_ctx(&ctx);
    if (st != PDZ_OK) return st;
    return launch_rank(ctx->binom, n_sites, n, bits, count, ranks, ctx->err, (hipStream_t)stream);
}

pdz_status pdz_unrank(int32_t n_sites, int32_t n, const uint32_t* ranks, uint64_t count, uint32_t* bits,
                      void* stream) {
    g_last_error.clear();
    if (n_sites < 1 || n_sites > kMaxSites) return fail(PDZ_ERANGE, "n_sites must be in [1, 32]");
    if (n < 0 || n > n_sites) return fail(PDZ_EINVAL, "n must be in [0, n_sites]");
    if (count > 0 && (!bits || !ranks)) return fail(PDZ_EINVAL, "NULL array");
    DeviceCtx* ctx = nullptr;
    pdz_status st = device_ctx(&ctx);
    if (st != PDZ_OK) return st;
    return launch_unrank(ctx->binom, n_sites, n, ranks, count, bits, ctx->err, (hipStream_t)stream);
}

pdz_status pdz_device_errors(uint32_t* word) {
    g_last_error.clear();
    DeviceCtx* ctx = nullptr;
    pdz_status st = device_ctx(&ctx);
    if (st != PDZ_OK) return st;
    PDZ_HIP(hipDeviceSynchronize());
    uint32_t w = 0;
    PDZ_HIP(hipMemcpy(&w, ctx->err, sizeof(w), hipMemcpyDeviceToHost));
    PDZ_HIP(hipMemset(ctx->err, 0, sizeof(uint32_t)));
    if (word) *word = w;
    if (w) return fail(PDZ_EDEVICE, "device error word " + std::to_string(w));
    return ok();
}

pdz_status pdz_hv(pdz_problem p, pdz_dtype dt, const void* x, void* y, void* stream) {
    g_last_error.clear();
    if (!p) return fail(PDZ_EINVAL, "problem is NULL");
    if (dt != PDZ_F64 && dt != PDZ_F32) return fail(PDZ_EINVAL, "dtype must be PDZ_F64 or PDZ_F32");
    if (!x || !y) return fail(PDZ_EINVAL, "NULL vector");
    const size_t bytes = (size_t)p->D * (dt == PDZ_F64 ? 8 : 4);
    const char* xb = static_cast<const char*>(x);
    const char* yb = static_cast<const char*>(y);
    if (xb < yb + bytes && yb < xb + bytes) return fail(PDZ_EINVAL, "x and y overlap");
    int dev = 0;
    PDZ_HIP(hipGetDevice(&dev));
    if (dev != p->device) return fail(PDZ_EINVAL, "problem lives on another device");
    return launch_hv_any(p, dt, x, y, (hipStream_t)stream);
}

pdz_status pdz_hv_pitched(pdz_problem p, pdz_dtype dt, const void* x, void* y, uint64_t pitch, void* stream) {
    g_last_error.clear();
    if (!p) return fail(PDZ_EINVAL, "problem is NULL");
    if (dt != PDZ_F64 && dt != PDZ_F32) return fail(PDZ_EINVAL, "dtype must be PDZ_F64 or PDZ_F32");
    if (!x || !y) return fail(PDZ_EINVAL, "NULL vector");
    if (pitch < p->dn.D) return fail(PDZ_EINVAL, "pitch shorter than a row");
    if ((p->ks || p->par || p->hv_path != 0) && pitch != p->dn.D)
        return fail(PDZ_EINVAL, "padded rows need a real-space problem with hop tables");
    const size_t bytes = (size_t)(p->up.D * pitch) * (dt == PDZ_F64 ? 8 : 4);
    const char* xb = static_cast<const char*>(x);
    const char* yb = static_cast<const char*>(y);
    if (xb < yb + bytes && yb < xb + bytes) return fail(PDZ_EINVAL, "x and y overlap");
    int dev = 0;
    PDZ_HIP(hipGetDevice(&dev));
    if (dev != p->device) return fail(PDZ_EINVAL, "problem lives on another device");
    return launch_hv_any(p, dt, x, y, (hipStream_t)stream, nullptr, kPassDown | kPassUp, nullptr,
                         pitch == p->dn.D ? 0 : pitch);
}

}  // extern "C"
