// extern "C" boundary: argument checks, error translation, data accessors.
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>
#include <string>

#include "hierarchy.h"
#include "server.h"

struct amg_hierarchy {
    std::unique_ptr<matamg::Hierarchy> h;
};

struct amg_server {
    std::unique_ptr<matamg::Server> s;
};

namespace matamg {

thread_local std::string g_last_error;
thread_local AllocMode g_alloc_mode;
AllocMode& alloc_mode() { return g_alloc_mode; }

void* readback_buffer() {
    thread_local void* buf = nullptr;
    if (!buf) MATAMG_HIP(hipHostMalloc(&buf, kReadbackBytes, hipHostMallocDefault));
    return buf;
}

namespace {
std::mutex g_idle_mu;
std::unordered_map<uint64_t, std::vector<void*>> g_idle;  // (device, bytes) -> buffers
uint64_t g_idle_bytes = 0;
std::mutex g_stream_mu;
std::vector<hipStream_t> g_streams[64];  // idle solve streams per device

uint64_t idle_key(size_t bytes) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    return ((uint64_t)(dev & 0xff) << 56) | (uint64_t)bytes;
}
}  // namespace

void* idle_take(size_t bytes) {
    const uint64_t key = idle_key(bytes);
    std::lock_guard<std::mutex> lock(g_idle_mu);
    auto it = g_idle.find(key);
    if (it == g_idle.end() || it->second.empty()) return nullptr;
    void* p = it->second.back();
    it->second.pop_back();
    g_idle_bytes -= bytes;
    return p;
}

bool idle_put(void* p, size_t bytes) {
    const uint64_t key = idle_key(bytes);
    std::lock_guard<std::mutex> lock(g_idle_mu);
    if (g_idle_bytes + bytes > kIdleCacheBytes) return false;
    g_idle[key].push_back(p);
    g_idle_bytes += bytes;
    return true;
}

namespace {
std::mutex g_temp_mu;
std::unordered_map<hipStream_t, std::unordered_map<size_t, std::vector<void*>>> g_temps;
uint64_t g_temp_bytes = 0;
}  // namespace

void* stream_take(hipStream_t st, size_t bytes) {
    std::lock_guard<std::mutex> lock(g_temp_mu);
    auto it = g_temps.find(st);
    if (it == g_temps.end()) return nullptr;
    auto jt = it->second.find(bytes);
    if (jt == it->second.end() || jt->second.empty()) return nullptr;
    void* p = jt->second.back();
    jt->second.pop_back();
    g_temp_bytes -= bytes;
    return p;
}

bool stream_put(hipStream_t st, void* p, size_t bytes) {
    std::lock_guard<std::mutex> lock(g_temp_mu);
    if (g_temp_bytes + bytes > kIdleCacheBytes) return false;
    g_temps[st][bytes].push_back(p);
    g_temp_bytes += bytes;
    return true;
}

void stream_cache_flush(hipStream_t st, bool to_idle) {
    std::unordered_map<size_t, std::vector<void*>> mine;
    {
        std::lock_guard<std::mutex> lock(g_temp_mu);
        auto it = g_temps.find(st);
        if (it == g_temps.end()) return;
        mine.swap(it->second);
        g_temps.erase(it);
        for (auto& kv : mine) g_temp_bytes -= kv.first * kv.second.size();
    }
    for (auto& kv : mine)
        for (void* p : kv.second)
            if (!(to_idle && idle_put(p, kv.first))) (void)hipFreeAsync(p, st);
}

uint64_t idle_trim(hipStream_t st) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    const uint64_t mine = (uint64_t)(dev & 0xff) << 56;
    std::vector<std::pair<void*, size_t>> out;
    {
        std::lock_guard<std::mutex> lock(g_idle_mu);
        for (auto it = g_idle.begin(); it != g_idle.end();) {
            if ((it->first & (0xffull << 56)) == mine) {
                const size_t bytes = (size_t)(it->first & ((1ull << 56) - 1));
                for (void* p : it->second) out.emplace_back(p, bytes);
                g_idle_bytes -= bytes * it->second.size();
                it = g_idle.erase(it);
            } else {
                ++it;
            }
        }
    }
    uint64_t total = 0;
    for (auto& pb : out) {
        (void)hipFreeAsync(pb.first, st);
        total += pb.second;
    }
    return total;
}

hipStream_t take_stream() {
    int dev = 0;
    MATAMG_HIP(hipGetDevice(&dev));
    {
        std::lock_guard<std::mutex> lock(g_stream_mu);
        if (dev >= 0 && dev < 64 && !g_streams[dev].empty()) {
            hipStream_t st = g_streams[dev].back();
            g_streams[dev].pop_back();
            return st;
        }
    }
    hipStream_t st = nullptr;
    MATAMG_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    return st;
}

void give_stream(hipStream_t st) {
    if (!st) return;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipStreamDestroy(st);
        return;
    }
    std::lock_guard<std::mutex> lock(g_stream_mu);
    g_streams[dev].push_back(st);
}

hipStream_t release_stream() {
    static hipStream_t streams[64] = {nullptr};
    static std::mutex mu;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
        streams[dev] = nullptr;
    return streams[dev];
}

bool pool_enabled() {
    const char* e = std::getenv("MATAMG_NO_POOL");
    return !(e && e[0] == '1');
}

void keep_pool_memory(int device) {
    hipMemPool_t pool = nullptr;
    MATAMG_HIP(hipDeviceGetDefaultMemPool(&pool, device));
    uint64_t keep = UINT64_MAX;
    MATAMG_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
}

[[noreturn]] void fail(amg_status code, const std::string& msg) { throw Error{code, msg}; }

}  // namespace matamg

using namespace matamg;

namespace {

template <typename F>
amg_status guarded(F&& f) {
    try {
        g_last_error.clear();
        return f();
    } catch (const Error& e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return AMG_ERR_OUT_OF_MEMORY;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return AMG_ERR_HIP;
    } catch (...) {
        g_last_error = "unknown failure";
        return AMG_ERR_HIP;
    }
}

amg_status check_options(const amg_options& o) {
    if (o.dim < 1 || o.dim > 3) fail(AMG_ERR_INVALID_ARG, "dim must be 1, 2 or 3");
    if (!(o.theta >= 0.0 && o.theta <= 1.0)) fail(AMG_ERR_INVALID_ARG, "theta must lie in [0, 1]");
    if (o.soc < AMG_SOC_MATERIAL || o.soc > AMG_SOC_SA) fail(AMG_ERR_INVALID_ARG, "unknown strength measure");
    if (o.drop != AMG_DROP_POINTWISE && o.drop != AMG_DROP_CUT) fail(AMG_ERR_INVALID_ARG, "unknown dropping criterion");
    if (o.smoother != AMG_SMOOTH_CHEBYSHEV && o.smoother != AMG_SMOOTH_JACOBI && o.smoother != AMG_SMOOTH_JACOBI_SCALED)
        fail(AMG_ERR_INVALID_ARG, "unknown smoother");
    if (!(o.jacobi_omega > 0.0) || !std::isfinite(o.jacobi_omega))
        fail(AMG_ERR_INVALID_ARG, "jacobi_omega must be positive and finite");
    if (o.max_coarse < 1) fail(AMG_ERR_INVALID_ARG, "max_coarse must be positive");
    if (o.max_coarse > 20000) fail(AMG_ERR_INVALID_ARG, "max_coarse above 20000 (dense coarse solve)");
    if (o.max_levels < 1 || o.max_levels > 16) fail(AMG_ERR_INVALID_ARG, "max_levels must lie in [1, 16]");
    if (o.cheb_degree < 1 || o.cheb_degree > 8) fail(AMG_ERR_INVALID_ARG, "cheb_degree must lie in [1, 8]");
    if (!(o.cheb_ratio > 1.0) || !(o.cheb_boost > 0.0)) fail(AMG_ERR_INVALID_ARG, "bad Chebyshev interval");
    if (o.power_iters < 1 || o.power_iters > 1000) fail(AMG_ERR_INVALID_ARG, "power_iters must lie in [1, 1000]");
    if (o.jacobi_sweeps < 1 || o.jacobi_sweeps > 8) fail(AMG_ERR_INVALID_ARG, "jacobi_sweeps must lie in [1, 8]");
    if (o.precision != AMG_PREC_FP64 && o.precision != AMG_PREC_FP32_HIER)
        fail(AMG_ERR_INVALID_ARG, "unknown precision");
    return AMG_OK;
}

Hierarchy& H(amg_hierarchy* h) {
    if (!h || !h->h) fail(AMG_ERR_INVALID_ARG, "null hierarchy");
    return *h->h;
}
const Hierarchy& H(const amg_hierarchy* h) {
    if (!h || !h->h) fail(AMG_ERR_INVALID_ARG, "null hierarchy");
    return *h->h;
}

}  // namespace

extern "C" {

amg_status amg_options_default(amg_options* o) {
    if (!o) return AMG_ERR_INVALID_ARG;
    std::memset(o, 0, sizeof(*o));
    o->dim = 3;
    o->theta = 0.08;
    o->soc = AMG_SOC_MATERIAL;
    o->drop = AMG_DROP_POINTWISE;
    o->smoother = AMG_SMOOTH_CHEBYSHEV;
    o->max_coarse = 5000;
    o->max_levels = 10;
    o->cheb_degree = 2;
    o->cheb_ratio = 30.0;
    o->cheb_boost = 1.1;
    o->power_iters = 10;
    o->omega_sym = 4.0 / 3.0;
    o->jacobi_omega = 2.0 / 3.0;
    o->jacobi_sweeps = 2;
    o->precision = AMG_PREC_FP64;
    o->seed = 0;
    return AMG_OK;
}

amg_status amg_setup(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val, int64_t nelem,
                     int32_t nodes_per_elem, const int32_t* elem_nodes, const double* elem_sigma,
                     const double* coords, const amg_options* opt, amg_ptr_kind kind, void* hip_stream,
                     amg_hierarchy** out) {
    return guarded([&]() -> amg_status {
        if (!out) fail(AMG_ERR_INVALID_ARG, "out is null");
        *out = nullptr;
        amg_options o;
        if (opt) o = *opt;
        else amg_options_default(&o);
        check_options(o);
        if (n <= 0 || n >= (int64_t)1 << 31) fail(AMG_ERR_INVALID_ARG, "n must lie in [1, 2^31)");
        if (!rowptr || !col || !val || !coords) fail(AMG_ERR_INVALID_ARG, "null CSR or coordinate array");
        if (nelem < 0 || (nelem > 0 && (!elem_nodes || !elem_sigma || nodes_per_elem <= 0)))
            fail(AMG_ERR_INVALID_ARG, "bad element arrays");
        if (kind != AMG_PTR_HOST && kind != AMG_PTR_DEVICE) fail(AMG_ERR_INVALID_ARG, "bad pointer kind");
        if (kind == AMG_PTR_HOST) {
            if (rowptr[0] != 0) fail(AMG_ERR_INVALID_ARG, "rowptr[0] must be 0");
            for (int64_t i = 0; i < n; ++i)
                if (rowptr[i + 1] < rowptr[i]) fail(AMG_ERR_INVALID_ARG, "rowptr is not non-decreasing");
        }
        hipStream_t s = (hipStream_t)hip_stream;
        auto h = build_hierarchy(n, rowptr, col, val, nelem, nodes_per_elem, elem_nodes, elem_sigma, coords, o,
                                 kind == AMG_PTR_HOST, s);
        auto* wrap = new amg_hierarchy{std::move(h)};
        *out = wrap;
        return AMG_OK;
    });
}

amg_status amg_pcg_solve(amg_hierarchy* hh, const double* b, double* x, double tol, int32_t max_iter,
                         amg_ptr_kind kind, void* hip_stream, amg_solve_info* info) {
    return guarded([&]() -> amg_status {
        Hierarchy& h = H(hh);
        if (!b || !x) fail(AMG_ERR_INVALID_ARG, "null b or x");
        if (!(tol > 0.0) || max_iter < 0) fail(AMG_ERR_INVALID_ARG, "tol must be positive, max_iter >= 0");
        return pcg_solve(h, b, x, tol, max_iter, kind == AMG_PTR_HOST, (hipStream_t)hip_stream, info);
    });
}

amg_status amg_pcg_solve_noalloc(amg_hierarchy* hh, const double* b, double* x, double tol, int32_t max_iter,
                                 void* hip_stream, amg_solve_info* info) {
    return guarded([&]() -> amg_status {
        Hierarchy& h = H(hh);
        if (!b || !x) fail(AMG_ERR_INVALID_ARG, "null b or x");
        if (!(tol > 0.0) || max_iter < 0) fail(AMG_ERR_INVALID_ARG, "tol must be positive, max_iter >= 0");
        return pcg_solve_noalloc(h, b, x, tol, max_iter, (hipStream_t)hip_stream, info);
    });
}

amg_status amg_update_values(amg_hierarchy* hh, const double* val, amg_ptr_kind kind, void* hip_stream) {
    return guarded([&]() -> amg_status {
        Hierarchy& h = H(hh);
        if (!val) fail(AMG_ERR_INVALID_ARG, "null values");
        if (kind != AMG_PTR_HOST && kind != AMG_PTR_DEVICE) fail(AMG_ERR_INVALID_ARG, "bad pointer kind");
        update_values(h, val, kind == AMG_PTR_HOST, (hipStream_t)hip_stream);
        return AMG_OK;
    });
}

amg_status amg_vcycle(amg_hierarchy* hh, const double* r, double* z, void* hip_stream) {
    return guarded([&]() -> amg_status {
        Hierarchy& h = H(hh);
        if (!r || !z) fail(AMG_ERR_INVALID_ARG, "null vector");
        h.vcycle(r, z, h.dt(S_TMP), (hipStream_t)hip_stream);
        return AMG_OK;
    });
}

amg_status amg_level_spmv(amg_hierarchy* hh, int32_t level, const double* x, double* y, void* hip_stream) {
    return guarded([&]() -> amg_status {
        Hierarchy& h = H(hh);
        if (level < 0 || level >= h.nlev) fail(AMG_ERR_INVALID_ARG, "level out of range");
        if (!x || !y) fail(AMG_ERR_INVALID_ARG, "null vector");
        const DCsr& A = h.lev[level].A;
        if (A.nblk <= 0) fail(AMG_ERR_INVALID_ARG, "level has no streaming layout");
        spmv<double>(A, A.val.get(), x, y, (hipStream_t)hip_stream);
        return AMG_OK;
    });
}

amg_status amg_hierarchy_info(const amg_hierarchy* hh, amg_hierarchy_stats* st) {
    return guarded([&]() -> amg_status {
        const Hierarchy& h = H(hh);
        if (!st) fail(AMG_ERR_INVALID_ARG, "null stats");
        std::memset(st, 0, sizeof(*st));
        st->levels = h.nlev;
        double tot = 0.0;
        for (int l = 0; l < h.nlev; ++l) {
            const Level& L = h.lev[l];
            st->n[l] = L.A.n;
            st->nnz[l] = L.A.nnz;
            st->nnz_p[l] = (l + 1 < h.nlev) ? L.P.nnz : 0;
            st->mis_rounds[l] = L.mis_rounds;
            st->omega[l] = L.omega;
            st->lam_pf[l] = L.lam_pf;
            st->lam_cheb[l] = L.lam_cheb;
            tot += (double)L.A.nnz;
        }
        st->op_complexity = tot / (double)h.lev[0].A.nnz;
        st->vcycle_alg_bytes = h.vcycle_alg_bytes();
        st->t_setup_s = h.t_setup;
        st->device_bytes = h.mem.bytes;
        st->device_peak_bytes = h.mem.peak;
        st->t_update_s = h.t_update;
        return AMG_OK;
    });
}

amg_status amg_get_aggregates(const amg_hierarchy* hh, int32_t level, int32_t* agg) {
    return guarded([&]() -> amg_status {
        const Hierarchy& h = H(hh);
        if (level < 0 || level + 1 >= h.nlev || !agg) fail(AMG_ERR_INVALID_ARG, "level out of range");
        MATAMG_HIP(hipMemcpy(agg, h.lev[level].agg.get(), sizeof(int) * (size_t)h.lev[level].A.n,
                             hipMemcpyDeviceToHost));
        return AMG_OK;
    });
}

amg_status amg_get_soc_mask(const amg_hierarchy* hh, int32_t level, uint8_t* mask) {
    return guarded([&]() -> amg_status {
        const Hierarchy& h = H(hh);
        if (level < 0 || level + 1 >= h.nlev || !mask) fail(AMG_ERR_INVALID_ARG, "level out of range");
        MATAMG_HIP(hipMemcpy(mask, h.lev[level].mask.get(), (size_t)h.lev[level].A.nnz, hipMemcpyDeviceToHost));
        return AMG_OK;
    });
}

amg_status amg_get_level_csr(const amg_hierarchy* hh, int32_t level, int32_t which, int32_t* rowptr,
                             int32_t* col, double* val) {
    return guarded([&]() -> amg_status {
        const Hierarchy& h = H(hh);
        if (level < 0 || level >= h.nlev) fail(AMG_ERR_INVALID_ARG, "level out of range");
        if (which < 0 || which > 2 || (which > 0 && level + 1 >= h.nlev))
            fail(AMG_ERR_INVALID_ARG, "no such matrix on this level");
        const Level& L = h.lev[level];
        const DCsr& M = which == 0 ? L.A : (which == 1 ? L.P : L.R);
        if (rowptr) MATAMG_HIP(hipMemcpy(rowptr, M.rowptr.get(), sizeof(int) * ((size_t)M.n + 1), hipMemcpyDeviceToHost));
        if (col) MATAMG_HIP(hipMemcpy(col, M.col.get(), sizeof(int) * (size_t)M.nnz, hipMemcpyDeviceToHost));
        if (val) MATAMG_HIP(hipMemcpy(val, M.val.get(), sizeof(double) * (size_t)M.nnz, hipMemcpyDeviceToHost));
        return AMG_OK;
    });
}

amg_status amg_get_level_aux(const amg_hierarchy* hh, int32_t level, int32_t which, double* out) {
    return guarded([&]() -> amg_status {
        const Hierarchy& h = H(hh);
        if (level < 0 || level >= h.nlev || !out) fail(AMG_ERR_INVALID_ARG, "level out of range");
        const Level& L = h.lev[level];
        const int dim = h.opt.dim, ncomp = dim * (dim + 1) / 2;
        if (which == 0) {
            MATAMG_HIP(hipMemcpy(out, L.x.get(), sizeof(double) * (size_t)L.A.n * dim, hipMemcpyDeviceToHost));
        } else if (which == 1) {
            MATAMG_HIP(hipMemcpy(out, L.sig.get(), sizeof(double) * (size_t)L.A.n * ncomp, hipMemcpyDeviceToHost));
        } else if (which == 2) {
            if (!L.dir) fail(AMG_ERR_INVALID_ARG, "no Dirichlet flags on this level");
            std::vector<uint8_t> d((size_t)L.A.n);
            MATAMG_HIP(hipMemcpy(d.data(), L.dir.get(), d.size(), hipMemcpyDeviceToHost));
            for (size_t i = 0; i < d.size(); ++i) out[i] = d[i];
        } else if (which == 3) {
            if (!L.S) fail(AMG_ERR_INVALID_ARG, "no strength values on this level");
            MATAMG_HIP(hipMemcpy(out, L.S.get(), sizeof(double) * (size_t)L.A.nnz, hipMemcpyDeviceToHost));
        } else {
            fail(AMG_ERR_INVALID_ARG, "unknown aux array");
        }
        return AMG_OK;
    });
}

amg_status amg_time_smoother(amg_hierarchy* hh, int32_t level, int32_t reps, void* hip_stream, double* avg_ms,
                             double* bytes_per_launch) {
    return guarded([&]() -> amg_status {
        Hierarchy& h = H(hh);
        if (level < 0 || level + 1 >= h.nlev) fail(AMG_ERR_INVALID_ARG, "level has no smoother");
        if (reps < 1 || !avg_ms) fail(AMG_ERR_INVALID_ARG, "reps must be positive");
        *avg_ms = h.time_smoother(level, reps, (hipStream_t)hip_stream, bytes_per_launch);
        return AMG_OK;
    });
}

void amg_free(amg_hierarchy* h) {
    if (!h) return;
    // let every stream of the device finish with the buffers; the pooled ones
    // are then idle and kept for reuse (those beyond the cache's limit go back
    // to the pool on a stream of the library's own)
    (void)hipDeviceSynchronize();
    try {
        hipStream_t fs = release_stream();
        {
            // the device is idle: its buffers are kept for the next hierarchy
            AllocStreamScope scope(fs, true);
            alloc_mode().idle = true;
            delete h;
        }
        if (fs) (void)hipStreamSynchronize(fs);
    } catch (...) {
    }
}

amg_status amg_trim_cache(int64_t* bytes) {
    return guarded([&]() -> amg_status {
        MATAMG_HIP(hipDeviceSynchronize());
        hipStream_t fs = release_stream();
        const uint64_t b = idle_trim(fs);
        if (fs) MATAMG_HIP(hipStreamSynchronize(fs));
        if (bytes) *bytes = (int64_t)b;
        return AMG_OK;
    });
}

// ------------------------------------------------------------------ serving
amg_status amg_server_create(const amg_options* opt, int64_t budget_bytes, int32_t max_active, int32_t setup_workers,
                             amg_server** out) {
    return guarded([&]() -> amg_status {
        if (!out) fail(AMG_ERR_INVALID_ARG, "out is null");
        *out = nullptr;
        amg_options o;
        if (opt) o = *opt;
        else amg_options_default(&o);
        check_options(o);
        if (budget_bytes <= 0) fail(AMG_ERR_INVALID_ARG, "budget must be positive");
        if (max_active < 1 || max_active > 1024) fail(AMG_ERR_INVALID_ARG, "max_active must lie in [1, 1024]");
        if (setup_workers < 1 || setup_workers > 8) fail(AMG_ERR_INVALID_ARG, "setup_workers must lie in [1, 8]");
        auto srv = std::make_unique<Server>(o, budget_bytes, max_active, setup_workers);
        *out = new amg_server{std::move(srv)};
        return AMG_OK;
    });
}

amg_status amg_server_submit(amg_server* s, int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                             int64_t nelem, int32_t nodes_per_elem, const int32_t* elem_nodes,
                             const double* elem_sigma, const double* coords, const double* b, const double* x0,
                             double tol, int32_t max_iter, uint64_t* request_id) {
    return guarded([&]() -> amg_status {
        if (!s || !s->s) fail(AMG_ERR_INVALID_ARG, "null server");
        return s->s->submit(n, rowptr, col, val, nelem, nodes_per_elem, elem_nodes, elem_sigma, coords, b, x0, tol,
                            max_iter, request_id);
    });
}

amg_status amg_server_poll(amg_server* s, double timeout_s, uint64_t* ids, int32_t cap, int32_t* ndone) {
    return guarded([&]() -> amg_status {
        if (!s || !s->s || !ndone || cap < 0 || (cap > 0 && !ids)) fail(AMG_ERR_INVALID_ARG, "bad poll arguments");
        *ndone = s->s->poll(ids, cap, timeout_s);
        return AMG_OK;
    });
}

amg_status amg_server_result(amg_server* s, uint64_t id, double* x, amg_solve_info* info, amg_request_stats* rs) {
    return guarded([&]() -> amg_status {
        if (!s || !s->s) fail(AMG_ERR_INVALID_ARG, "null server");
        std::unique_ptr<Request> r = s->s->take(id);
        if (!r) fail(AMG_ERR_INVALID_ARG, "request " + std::to_string(id) + " is unknown, unfinished or already taken");
        if (x && !r->x.empty()) std::memcpy(x, r->x.data(), sizeof(double) * r->x.size());
        if (info) {
            info->iterations = r->iters;
            info->rel_res_true = r->rel_true;
            info->t_solve_s = r->t_done - r->t_setup_done;
            info->status = r->status;
        }
        if (rs) {
            std::memset(rs, 0, sizeof(*rs));
            rs->t_arrival = r->t_arrival;
            rs->t_admit = r->t_admit;
            rs->t_setup_done = r->t_setup_done;
            rs->t_done = r->t_done;
            rs->est_bytes = r->est;
            rs->setup_peak_bytes = r->setup_peak;
            rs->resident_bytes = r->resident;
            rs->levels = r->levels;
            rs->max_batch = r->max_batch;
            rs->n = r->n;
            rs->nnz = r->nnz;
        }
        if (r->status != AMG_OK && !r->error.empty()) g_last_error = r->error;
        return AMG_OK;
    });
}

amg_status amg_server_info(amg_server* s, amg_server_stats* out) {
    return guarded([&]() -> amg_status {
        if (!s || !s->s || !out) fail(AMG_ERR_INVALID_ARG, "bad stats arguments");
        ServerStats st;
        int active = 0;
        int64_t budget = 0, used = 0, peak = 0, waiting = 0;
        s->s->stats(&st, &budget, &used, &peak, &active, &waiting);
        std::memset(out, 0, sizeof(*out));
        out->submitted = st.submitted;
        out->completed = st.completed;
        out->failed = st.failed;
        out->rejected = st.rejected;
        out->budget_bytes = budget;
        out->reserved_bytes = used;
        out->peak_reserved_bytes = peak;
        out->active = active;
        out->waiting = waiting;
        out->steps = st.steps;
        out->launches = st.launches;
        out->mean_batch = st.steps > 0 ? (double)st.batch_sum / (double)st.steps : 0.0;
        out->max_batch = st.max_batch;
        out->estimate_exceeded = st.estimate_exceeded;
        return AMG_OK;
    });
}

amg_status amg_server_set_batch_wait(amg_server* s, double seconds) {
    return guarded([&]() -> amg_status {
        if (!s || !s->s) fail(AMG_ERR_INVALID_ARG, "null server");
        if (!(seconds >= 0.0 && seconds <= 10.0)) fail(AMG_ERR_INVALID_ARG, "batch wait must lie in [0, 10] s");
        s->s->set_batch_wait(seconds);
        return AMG_OK;
    });
}

void amg_server_destroy(amg_server* s) {
    try {
        delete s;
    } catch (...) {
    }
}

const char* amg_status_string(amg_status s) {
    switch (s) {
        case AMG_OK: return "ok";
        case AMG_ERR_INVALID_ARG: return "invalid argument";
        case AMG_ERR_OUT_OF_MEMORY: return "out of memory";
        case AMG_ERR_HIP: return "HIP runtime error";
        case AMG_ERR_NOT_SPD: return "not symmetric positive definite";
        case AMG_ERR_COARSENING_STAGNATED: return "coarsening stagnated";
        case AMG_ERR_NOT_CONVERGED: return "not converged";
        case AMG_ERR_BREAKDOWN: return "CG breakdown";
        case AMG_ERR_BUDGET: return "request exceeds the memory budget";
    }
    return "unknown status";
}

const char* amg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
