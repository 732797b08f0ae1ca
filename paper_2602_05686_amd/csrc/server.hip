// Solve server (see server.h).
//
// Threads: `setup_workers` setup threads, each with its own stream, build
// the hierarchies of admitted requests; one engine thread owns the engine
// stream and advances every solving request by one preconditioned CG step
// per round.  A round is one sequence of batched launches: for each step of
// the V-cycle (pre-smoothing, residual and restriction per level going down,
// the dense coarsest solve, prolongation and post-smoothing per level going
// up) and of the CG update, one launch covers that step for every request
// that has it (requests of different depths take part in the levels they
// have).  The per-request argument records of a round are built on the
// host, uploaded with one copy, and read by the launches.  Each request's
// blocks compute exactly what its one-hierarchy launches compute, and its
// CG control follows the one-hierarchy solver step for step, so a result
// does not depend on the other requests in flight.
//
// Device memory: threads allocate from the device's stream-ordered pool on
// their own stream (AllocStreamScope), so building and freeing hierarchies
// never waits for the other streams.  Admission reserves a request's
// estimated setup peak (admission.h) until its setup ends, then only the
// bytes its hierarchy keeps.
#include "server.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <type_traits>

#include "batch.h"

namespace matamg {
namespace {

double wall_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

template <typename T>
struct LV;
template <>
struct LV<double> {
    static double* b(Level& L) { return L.b.get(); }
    static double* xa(Level& L) { return L.xa.get(); }
    static double* xb(Level& L) { return L.xb.get(); }
    static double* d(Level& L) { return L.d.get(); }
    static double* r(Level& L) { return L.r.get(); }
    static const double* A(const DCsr& M) { return M.val.get(); }
    static const double* dinv(Level& L) { return L.dinv.get(); }
};
template <>
struct LV<float> {
    static float* b(Level& L) { return L.fb.get(); }
    static float* xa(Level& L) { return L.fxa.get(); }
    static float* xb(Level& L) { return L.fxb.get(); }
    static float* d(Level& L) { return L.fd.get(); }
    static float* r(Level& L) { return L.fr.get(); }
    static const float* A(const DCsr& M) { return M.val32.get(); }
    static const float* dinv(Level& L) { return L.dinv32.get(); }
};

template <typename T>
SArgs<T> sargs(const DCsr& M, const T* val, const T* x) {
    // the batched streaming kernels stage kStreamCap entries per block; the
    // server's hierarchies keep that partition
    if (M.cap != kStreamCap) fail(AMG_ERR_HIP, "served matrix has widened streaming blocks");
    SArgs<T> a{};
    a.rowptr = M.rowptr.get();
    a.col = M.col.get();
    a.col16 = M.col16.get();
    a.cbase = M.cbase.get();
    a.val = val;
    a.blk = M.blk.get();
    a.blkk = M.blkk.get();
    a.ustart = M.ustart.get();
    a.uoff = M.uoff.get();
    a.urun = M.urun.get();
    a.x = x;
    return a;
}

enum Kind { K_NONE, K_STREAM, K_STREAM64, K_SFIRST, K_GEMV, K_CGDIR, K_CGUPD, K_FINISH, K_SINGLE };

// one batched launch position of a round
template <typename T>
struct Stage {
    int kind = K_NONE;
    int mode = 0;
    bool dot = false;
    std::vector<SArgs<T>> s[2];  // by threads per row: 1, 8
    std::vector<SArgs<double>> d[2];
    std::vector<int> sn[2];      // row blocks per record
    std::vector<SmoothFirstArgs<T>> sf;
    std::vector<GemvArgs<T>> gv;
    std::vector<CgDirArgs> cd;
    std::vector<CgUpdArgs> cu;
    std::vector<int> vn;         // blocks per record (vector and GEMV stages)
    std::vector<FinishArgs> fin;
    std::vector<std::pair<Request*, DotTarget>> single;
    size_t off_rec[2] = {0, 0}, off_st[2] = {0, 0};
    int nseg[2] = {0, 0}, total[2] = {0, 0};
};

// launch order of a round: down sweep by ascending level, coarsest solve,
// up sweep by descending level, then the CG update
int64_t key_down(int l, int j) { return ((int64_t)0 << 40) | ((int64_t)l << 20) | j; }
int64_t key_coarse(int j) { return ((int64_t)1 << 40) | j; }
int64_t key_up(int l, int j) { return ((int64_t)2 << 40) | ((int64_t)(15 - l) << 20) | j; }
int64_t key_cg(int j) { return ((int64_t)3 << 40) | j; }
constexpr int kDownResid = 1000, kDownRestrict = 1001, kUpFinish = 100000;

template <typename T>
Stage<T>& stage(std::map<int64_t, Stage<T>>& st, int64_t key, int kind, int mode = 0, bool dot = false) {
    Stage<T>& s = st[key];
    s.kind = kind;
    s.mode = mode;
    s.dot = dot;
    return s;
}

template <typename T>
void add_stream(Stage<T>& s, const DCsr& M, const SArgs<T>& a) {
    if (M.nblk <= 0) return;
    const int g = M.group == 1 ? 0 : 1;
    s.s[g].push_back(a);
    s.sn[g].push_back(M.nblk);
}

void add_stream64(Stage<float>& s, const DCsr& M, const SArgs<double>& a) {
    if (M.nblk <= 0) return;
    const int g = M.group == 1 ? 0 : 1;
    s.d[g].push_back(a);
    s.sn[g].push_back(M.nblk);
}
void add_stream64(Stage<double>& s, const DCsr& M, const SArgs<double>& a) {
    if (M.nblk <= 0) return;
    const int g = M.group == 1 ? 0 : 1;
    s.d[g].push_back(a);
    s.sn[g].push_back(M.nblk);
}

// The launches of one V-cycle z = M r of request R, in the order and with
// the operands of Hierarchy::vcycle_t, filed under their round positions.
template <typename T>
void emit_vcycle(std::map<int64_t, Stage<T>>& st, Request* R, DotTarget rz) {
    using V = LV<T>;
    Hierarchy& h = *R->h;
    const int L = h.nlev;
    double* r64 = h.cr.get();
    double* z64 = h.cz.get();
    if (L == 1) {
        stage<T>(st, key_coarse(1), K_SINGLE).single.push_back({R, rz});
        return;
    }
    T* cur[16];
    for (int l = 0; l + 1 < L; ++l) {
        Level& Lv = h.lev[l];
        const int n = Lv.A.n;
        T* b;
        const double* b64 = nullptr;
        if constexpr (std::is_same<T, double>::value) {
            b = (l == 0) ? r64 : V::b(Lv);
        } else {
            b = V::b(Lv);
            if (l == 0) b64 = r64;
        }
        T* x = V::xa(Lv);
        T* y = V::xb(Lv);
        {
            Stage<T>& s = stage<T>(st, key_down(l, 0), K_SFIRST);
            s.sf.push_back(SmoothFirstArgs<T>{n, b64, b, V::dinv(Lv), (T)Lv.c2[0], V::d(Lv), x});
            s.vn.push_back(vec_grid(n));
        }
        for (size_t k = 1; k < Lv.c1.size(); ++k) {
            SArgs<T> a = sargs<T>(Lv.A, V::A(Lv.A), x);
            a.b = b;
            a.yin = x;
            a.dinv = V::dinv(Lv);
            a.d = V::d(Lv);
            a.c1 = (T)Lv.c1[k];
            a.c2 = (T)Lv.c2[k];
            a.y = y;
            add_stream(stage<T>(st, key_down(l, (int)k), K_STREAM, M_SMOOTH, false), Lv.A, a);
            std::swap(x, y);
        }
        cur[l] = x;
        {
            SArgs<T> a = sargs<T>(Lv.A, V::A(Lv.A), x);
            a.b = b;
            a.y = V::r(Lv);
            add_stream(stage<T>(st, key_down(l, kDownResid), K_STREAM, M_RESID, false), Lv.A, a);
        }
        {
            SArgs<T> a = sargs<T>(Lv.R, V::A(Lv.R), V::r(Lv));
            a.y = V::b(h.lev[l + 1]);
            add_stream(stage<T>(st, key_down(l, kDownRestrict), K_STREAM, M_PLAIN, false), Lv.R, a);
        }
    }
    Level& Lc = h.lev[L - 1];
    {
        Stage<T>& s = stage<T>(st, key_coarse(0), K_GEMV);
        s.gv.push_back(GemvArgs<T>{h.nL, h.Ainv.get(), V::b(Lc), V::xa(Lc)});
        s.vn.push_back(gemv_grid(h.nL));
    }
    cur[L - 1] = V::xa(Lc);
    for (int l = L - 2; l >= 0; --l) {
        Level& Lv = h.lev[l];
        T* b;
        if constexpr (std::is_same<T, double>::value) b = (l == 0) ? r64 : V::b(Lv);
        else b = V::b(Lv);
        T* x = cur[l];
        T* y = (x == V::xa(Lv)) ? V::xb(Lv) : V::xa(Lv);
        {
            SArgs<T> a = sargs<T>(Lv.P, V::A(Lv.P), cur[l + 1]);
            a.yin = x;
            a.y = x;
            add_stream(stage<T>(st, key_up(l, 0), K_STREAM, M_ADD, false), Lv.P, a);
        }
        const size_t steps = Lv.c1.size();
        for (size_t k = 0; k < steps; ++k) {
            const bool last = (l == 0 && k + 1 == steps);
            T* out = y;
            double* out64 = nullptr;
            if (last) {
                if constexpr (std::is_same<T, double>::value) out = z64;
                else out64 = z64;
            }
            SArgs<T> a = sargs<T>(Lv.A, V::A(Lv.A), x);
            a.b = b;
            a.yin = x;
            a.dinv = V::dinv(Lv);
            a.d = V::d(Lv);
            a.c1 = (T)(k == 0 ? 0.0 : Lv.c1[k]);
            a.c2 = (T)Lv.c2[k];
            a.y = out;
            a.y64 = out64;
            a.dotvec = last ? r64 : nullptr;
            a.dt = last ? rz : DotTarget{};
            add_stream(stage<T>(st, key_up(l, 1 + 2 * (int)k + (last ? 1 : 0)), K_STREAM, M_SMOOTH, last), Lv.A, a);
            if (!last) std::swap(x, y);
        }
        cur[l] = x;
    }
    stage<T>(st, key_up(0, kUpFinish), K_FINISH).fin.push_back(FinishArgs{stream_partials(h.lev[0].A), rz.partial, rz.result});
}

struct TableBuilder {
    std::vector<unsigned char> buf;
    template <class R>
    size_t put(const std::vector<R>& v) {
        size_t off = (buf.size() + 63) & ~(size_t)63;
        buf.resize(off + v.size() * sizeof(R));
        if (!v.empty()) std::memcpy(buf.data() + off, v.data(), v.size() * sizeof(R));
        return off;
    }
};

std::vector<int> prefix(const std::vector<int>& cnt) {
    std::vector<int> s(cnt.size() + 1, 0);
    for (size_t i = 0; i < cnt.size(); ++i) s[i + 1] = s[i] + cnt[i];
    return s;
}

}  // namespace

// ---------------------------------------------------------------- server
Server::Server(const amg_options& opt, int64_t budget, int max_active, int setup_workers)
    : opt_(opt), max_active_(max_active), adm_(budget, max_active) {
    t0_ = wall_s();
    MATAMG_HIP(hipGetDevice(&device_));
    int pools = 0;
    MATAMG_HIP(hipDeviceGetAttribute(&pools, hipDeviceAttributeMemoryPoolsSupported, device_));
    if (!pools) fail(AMG_ERR_HIP, "the device has no stream-ordered memory pool");
    // keep freed pool memory for reuse instead of returning it at every sync
    keep_pool_memory(device_);
    MATAMG_HIP(hipStreamCreateWithFlags(&es_, hipStreamNonBlocking));
    sscal_.alloc((size_t)max_active * S_NSCAL);
    MATAMG_HIP(hipMemsetAsync(sscal_.get(), 0, sizeof(double) * (size_t)max_active * S_NSCAL, es_));
    MATAMG_HIP(hipHostMalloc((void**)&hsc_, sizeof(double) * (size_t)max_active * S_NSCAL, hipHostMallocDefault));
    MATAMG_HIP(hipStreamSynchronize(es_));
    for (int i = max_active - 1; i >= 0; --i) free_slots_.push_back(i);
    engine_ = std::thread([this] { engine_main(); });
    for (int i = 0; i < setup_workers; ++i) workers_.emplace_back([this] { worker_main(); });
}

Server::~Server() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_setup_.notify_all();
    cv_engine_.notify_all();
    cv_done_.notify_all();
    for (auto& t : workers_) t.join();
    if (engine_.joinable()) engine_.join();
    {
        AllocStreamScope scope(es_);
        reqs_.clear();
        dtab_.release();
        sscal_.release();
    }
    (void)hipStreamSynchronize(es_);
    if (hsc_) (void)hipHostFree(hsc_);
    if (htab_) (void)hipHostFree(htab_);
    (void)hipStreamDestroy(es_);
    hipMemPool_t pool = nullptr;
    if (hipDeviceGetDefaultMemPool(&pool, device_) == hipSuccess) (void)hipMemPoolTrimTo(pool, 0);
}

double Server::now() const { return wall_s() - t0_; }

amg_status Server::submit(int64_t n, const int* rowptr, const int* col, const double* val, int64_t nelem, int npe,
                          const int* elem_nodes, const double* elem_sigma, const double* coords, const double* b,
                          const double* x0, double tol, int max_iter, uint64_t* id) {
    const double t_arr = now();
    if (n <= 0 || n >= (int64_t)1 << 31 || !rowptr || !col || !val || !coords || !b || !id)
        fail(AMG_ERR_INVALID_ARG, "submit: missing arrays or bad n");
    if (nelem < 0 || (nelem > 0 && (npe <= 0 || !elem_nodes || !elem_sigma)))
        fail(AMG_ERR_INVALID_ARG, "submit: bad element arrays");
    if (!(tol > 0.0) || max_iter < 0) fail(AMG_ERR_INVALID_ARG, "submit: tol must be positive, max_iter >= 0");
    const int64_t nnz = rowptr[n];
    if (nnz < 0 || rowptr[0] != 0) fail(AMG_ERR_INVALID_ARG, "submit: bad row pointer");
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(b[i]) || (x0 && !std::isfinite(x0[i])))
            fail(AMG_ERR_INVALID_ARG, "submit: the right-hand side or the initial guess is not finite");
    const int dim = opt_.dim;
    const int64_t est = estimate_setup_bytes(n, nnz, nelem, npe, dim, opt_.max_coarse);
    if (!adm_.fits_ever(est)) {
        std::lock_guard<std::mutex> lk(mu_);
        st_.rejected++;
        fail(AMG_ERR_BUDGET, "request needs an estimated " + std::to_string(est) + " device bytes, above the budget of " +
                                 std::to_string(adm_.budget()));
    }
    auto R = std::make_unique<Request>();
    R->n = n;
    R->nnz = nnz;
    R->nelem = nelem;
    R->npe = npe;
    R->rowptr.assign(rowptr, rowptr + n + 1);
    R->col.assign(col, col + nnz);
    R->val.assign(val, val + nnz);
    if (nelem > 0) {
        R->elem_nodes.assign(elem_nodes, elem_nodes + nelem * npe);
        R->elem_sigma.assign(elem_sigma, elem_sigma + nelem * dim * dim);
    }
    R->coords.assign(coords, coords + n * dim);
    R->b.assign(b, b + n);
    if (x0) R->x0.assign(x0, x0 + n);
    R->tol = tol;
    R->max_iter = max_iter;
    R->est = est;
    R->t_arrival = t_arr;
    std::lock_guard<std::mutex> lk(mu_);
    R->id = next_id_++;
    *id = R->id;
    adm_.push(R->id, est);
    reqs_[R->id] = std::move(R);
    st_.submitted++;
    admit_locked();
    return AMG_OK;
}

void Server::set_batch_wait(double seconds) {
    std::lock_guard<std::mutex> lk(mu_);
    batch_wait_ = seconds;
}

void Server::admit_locked() {
    const double t = now();
    for (uint64_t id : adm_.admit()) {
        Request* R = reqs_.at(id).get();
        R->t_admit = t;
        setup_q_.push_back(R);
        ++in_setup_;
    }
    if (!setup_q_.empty()) cv_setup_.notify_all();
}

void Server::finish_locked(Request* R) {
    R->done = true;
    R->t_done = now();
    adm_.release(R->id);
    done_q_.push_back(R->id);
    admit_locked();
    cv_done_.notify_all();
}

int Server::poll(uint64_t* ids, int cap, double timeout_s) {
    std::unique_lock<std::mutex> lk(mu_);
    if (done_q_.empty() && timeout_s > 0.0)
        cv_done_.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return !done_q_.empty() || stop_; });
    int k = 0;
    while (k < cap && !done_q_.empty()) {
        ids[k++] = done_q_.front();
        done_q_.pop_front();
    }
    return k;
}

std::unique_ptr<Request> Server::take(uint64_t id) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(id);
    if (it == reqs_.end() || !it->second->done) return nullptr;
    std::unique_ptr<Request> r = std::move(it->second);
    reqs_.erase(it);
    return r;
}

void Server::stats(ServerStats* st, int64_t* budget, int64_t* used, int64_t* peak_used, int* active,
                   int64_t* waiting) {
    std::lock_guard<std::mutex> lk(mu_);
    *st = st_;
    *budget = adm_.budget();
    *used = adm_.used();
    *peak_used = adm_.peak_used();
    *active = adm_.active();
    *waiting = (int64_t)adm_.waiting();
}

// ----------------------------------------------------------- setup workers
void Server::worker_main() {
    hipStream_t s = nullptr;
    if (hipSetDevice(device_) != hipSuccess || hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess)
        return;
    {
        AllocStreamScope scope(s);
        for (;;) {
            Request* R = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_setup_.wait(lk, [&] { return stop_ || !setup_q_.empty(); });
                if (stop_) break;
                R = setup_q_.front();
                setup_q_.pop_front();
            }
            std::unique_ptr<Hierarchy> h;
            amg_status code = AMG_OK;
            std::string msg;
            try {
                h = build_hierarchy(R->n, R->rowptr.data(), R->col.data(), R->val.data(), R->nelem, R->npe,
                                    R->elem_nodes.data(), R->elem_sigma.data(), R->coords.data(), opt_, true, s, false);
                h->release_setup_data();
                MATAMG_HIP(hipStreamSynchronize(s));
            } catch (const Error& e) {
                code = e.code;
                msg = e.msg;
            } catch (const std::bad_alloc&) {
                code = AMG_ERR_OUT_OF_MEMORY;
                msg = "host allocation failed during setup";
            } catch (const std::exception& e) {
                code = AMG_ERR_HIP;
                msg = e.what();
            }
            if (code != AMG_OK) {
                h.reset();
                // copies from the inputs may still be queued after a failure
                (void)hipStreamSynchronize(s);
            }
            // the matrix and mesh inputs are on the device now
            std::vector<int>().swap(R->rowptr);
            std::vector<int>().swap(R->col);
            std::vector<int>().swap(R->elem_nodes);
            std::vector<double>().swap(R->val);
            std::vector<double>().swap(R->elem_sigma);
            std::vector<double>().swap(R->coords);
            std::lock_guard<std::mutex> lk(mu_);
            R->t_setup_done = now();
            --in_setup_;
            if (code != AMG_OK) {
                R->status = code;
                R->error = msg;
                st_.failed++;
                finish_locked(R);
            } else {
                R->setup_peak = h->mem.peak;
                R->levels = h->nlev;
                R->resident = h->mem.bytes + 8 * R->n;  // + the right-hand side kept by the engine
                if (R->setup_peak > R->est) st_.estimate_exceeded++;
                R->h = std::move(h);
                adm_.resize(R->id, R->resident);
                ready_.push_back(R);
                admit_locked();
            }
            cv_engine_.notify_one();  // a waiting engine counts the requests still in setup
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
}

// ------------------------------------------------------------------ engine
template <typename T>
void Server::run_step(std::vector<Request*>& batch) {
    std::map<int64_t, Stage<T>> st;
    for (Request* R : batch) {
        Hierarchy& h = *R->h;
        const DCsr& A = h.lev[0].A;
        const int n = A.n;
        double* sc = sscal_.get() + (size_t)R->slot * S_NSCAL;
        const int target = R->first ? R->cur : (R->cur == S_RZ0 ? S_RZ1 : S_RZ0);
        DotTarget rz{h.partial.get(), h.counter.get(), sc + target};
        emit_vcycle<T>(st, R, rz);
        {
            Stage<T>& s = stage<T>(st, key_cg(0), K_CGDIR);
            s.cd.push_back(CgDirArgs{n, h.cp.get(), h.cz.get(), sc + target, R->first ? nullptr : sc + R->cur});
            s.vn.push_back(vec_grid(n));
        }
        {
            SArgs<double> a = sargs<double>(A, A.val.get(), h.cp.get());
            a.y = h.cq.get();
            a.dt = DotTarget{h.partial.get(), h.counter.get(), sc + S_PQ};
            add_stream64(stage<T>(st, key_cg(1), K_STREAM64, M_DOTPQ, true), A, a);
        }
        stage<T>(st, key_cg(2), K_FINISH).fin.push_back(FinishArgs{stream_partials(A), h.partial.get(), sc + S_PQ});
        {
            Stage<T>& s = stage<T>(st, key_cg(3), K_CGUPD);
            s.cu.push_back(CgUpdArgs{n, h.cx.get(), h.cr.get(), h.cp.get(), h.cq.get(), sc + target, sc + S_PQ,
                                     h.partial.get()});
            s.vn.push_back(vec_grid(n));
        }
        stage<T>(st, key_cg(4), K_FINISH).fin.push_back(FinishArgs{vec_grid(n), h.partial.get(), sc + S_RR});
        R->max_batch = std::max<int>(R->max_batch, (int)batch.size());
    }
    // one table for the whole round
    TableBuilder tb;
    for (auto& kv : st) {
        Stage<T>& s = kv.second;
        for (int g = 0; g < 2; ++g) {
            if (s.sn[g].empty()) continue;
            s.off_rec[g] = (s.kind == K_STREAM64) ? tb.put(s.d[g]) : tb.put(s.s[g]);
            std::vector<int> pre = prefix(s.sn[g]);
            s.nseg[g] = (int)s.sn[g].size();
            s.total[g] = pre.back();
            s.off_st[g] = tb.put(pre);
        }
        if (!s.vn.empty()) {
            if (s.kind == K_SFIRST) s.off_rec[0] = tb.put(s.sf);
            else if (s.kind == K_GEMV) s.off_rec[0] = tb.put(s.gv);
            else if (s.kind == K_CGDIR) s.off_rec[0] = tb.put(s.cd);
            else if (s.kind == K_CGUPD) s.off_rec[0] = tb.put(s.cu);
            std::vector<int> pre = prefix(s.vn);
            s.nseg[0] = (int)s.vn.size();
            s.total[0] = pre.back();
            s.off_st[0] = tb.put(pre);
        }
        if (!s.fin.empty()) {
            s.off_rec[0] = tb.put(s.fin);
            s.nseg[0] = (int)s.fin.size();
        }
    }
    const size_t bytes = tb.buf.size();
    if (bytes > htab_cap_) {
        size_t cap = std::max<size_t>(bytes * 2, (size_t)1 << 20);
        if (htab_) (void)hipHostFree(htab_);
        htab_ = nullptr;
        htab_cap_ = 0;
        MATAMG_HIP(hipHostMalloc((void**)&htab_, cap, hipHostMallocDefault));
        htab_cap_ = cap;
        dtab_.alloc(cap);
    }
    std::memcpy(htab_, tb.buf.data(), bytes);
    MATAMG_HIP(hipMemcpyAsync(dtab_.get(), htab_, bytes, hipMemcpyHostToDevice, es_));
    unsigned char* base = dtab_.get();
    int64_t launches = 0;
    for (auto& kv : st) {
        Stage<T>& s = kv.second;
        switch (s.kind) {
            case K_STREAM:
                for (int g = 0; g < 2; ++g) {
                    if (!s.nseg[g]) continue;
                    stream_batch<T>(s.mode, s.dot, g == 0 ? 1 : 8, (const SArgs<T>*)(base + s.off_rec[g]),
                                    (const int*)(base + s.off_st[g]), s.nseg[g], s.total[g], es_);
                    ++launches;
                }
                break;
            case K_STREAM64:
                for (int g = 0; g < 2; ++g) {
                    if (!s.nseg[g]) continue;
                    stream_batch<double>(s.mode, s.dot, g == 0 ? 1 : 8, (const SArgs<double>*)(base + s.off_rec[g]),
                                         (const int*)(base + s.off_st[g]), s.nseg[g], s.total[g], es_);
                    ++launches;
                }
                break;
            case K_SFIRST:
                smooth_first_batch<T>((const SmoothFirstArgs<T>*)(base + s.off_rec[0]), (const int*)(base + s.off_st[0]),
                                      s.nseg[0], s.total[0], es_);
                ++launches;
                break;
            case K_GEMV:
                gemv_batch<T>((const GemvArgs<T>*)(base + s.off_rec[0]), (const int*)(base + s.off_st[0]), s.nseg[0],
                              s.total[0], es_);
                ++launches;
                break;
            case K_CGDIR:
                cg_direction_batch((const CgDirArgs*)(base + s.off_rec[0]), (const int*)(base + s.off_st[0]),
                                   s.nseg[0], s.total[0], es_);
                ++launches;
                break;
            case K_CGUPD:
                cg_update_batch((const CgUpdArgs*)(base + s.off_rec[0]), (const int*)(base + s.off_st[0]), s.nseg[0],
                                s.total[0], es_);
                ++launches;
                break;
            case K_FINISH:
                finish_batch((const FinishArgs*)(base + s.off_rec[0]), s.nseg[0], es_);
                ++launches;
                break;
            case K_SINGLE:
                // one-level hierarchies: the coarse solve is the whole V-cycle
                for (auto& p : s.single) p.first->h->vcycle(p.first->h->cr.get(), p.first->h->cz.get(), p.second, es_);
                launches += 2 * (int64_t)s.single.size();
                break;
            default:
                break;
        }
    }
    std::lock_guard<std::mutex> lk(mu_);
    st_.steps++;
    st_.launches += launches;
    st_.batch_sum += (int64_t)batch.size();
    st_.max_batch = std::max<int64_t>(st_.max_batch, (int64_t)batch.size());
}

void Server::engine_main() {
    if (hipSetDevice(device_) != hipSuccess) return;
    AllocStreamScope scope(es_);
    std::vector<Request*> solving;
    const size_t nsc = (size_t)max_active_ * S_NSCAL;
    auto read_scalars = [&]() {
        MATAMG_HIP(hipMemcpyAsync(hsc_, sscal_.get(), sizeof(double) * nsc, hipMemcpyDeviceToHost, es_));
        MATAMG_HIP(hipStreamSynchronize(es_));
    };
    auto sc = [&](Request* R, int k) { return hsc_[(size_t)R->slot * S_NSCAL + k]; };
    // hand the solution back and free the hierarchy
    auto complete = [&](Request* R, amg_status status) {
        const int n = (int)R->n;
        R->x.resize(n);
        d2h(R->x.data(), R->h->cx.get(), n, es_);
        R->status = status;
        R->h.reset();
        std::vector<double>().swap(R->b);
        std::vector<double>().swap(R->x0);
        free_slots_.push_back(R->slot);
        std::lock_guard<std::mutex> lk(mu_);
        st_.completed++;
        finish_locked(R);
    };
    auto fail_all = [&](std::vector<Request*>& rs, const Error& e) {
        for (Request* R : rs) {
            if (R->done) continue;
            R->h.reset();
            R->status = e.code;
            R->error = e.msg;
            if (R->slot >= 0) free_slots_.push_back(R->slot);
            std::lock_guard<std::mutex> lk(mu_);
            st_.failed++;
            finish_locked(R);
        }
        rs.clear();
    };
    for (;;) {
        std::vector<Request*> fresh;
        {
            std::unique_lock<std::mutex> lk(mu_);
            cv_engine_.wait(lk, [&] { return stop_ || !ready_.empty() || !solving.empty(); });
            if (stop_) break;
            if (solving.empty() && batch_wait_ > 0.0 && in_setup_ > 0) {
                // idle: give the requests still in setup a moment to join the first round
                const auto until = std::chrono::steady_clock::now() +
                                   std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                                       std::chrono::duration<double>(batch_wait_));
                cv_engine_.wait_until(lk, until, [&] { return stop_ || in_setup_ == 0; });
                if (stop_) break;
            }
            fresh.swap(ready_);
        }
        try {
            if (!fresh.empty()) {
                // initial residual of each new request, as the one-hierarchy solver computes it
                for (Request* R : fresh) {
                    Hierarchy& h = *R->h;
                    const DCsr& A = h.lev[0].A;
                    const int n = A.n;
                    R->slot = free_slots_.back();
                    free_slots_.pop_back();
                    double* s = sscal_.get() + (size_t)R->slot * S_NSCAL;
                    MATAMG_HIP(hipMemsetAsync(s, 0, sizeof(double) * S_NSCAL, es_));
                    if (!h.cb) h.cb.alloc(n, &h.mem);
                    h2d(h.cb.get(), R->b.data(), n, es_);
                    if (R->x0.empty()) MATAMG_HIP(hipMemsetAsync(h.cx.get(), 0, sizeof(double) * n, es_));
                    else h2d(h.cx.get(), R->x0.data(), n, es_);
                    dot<double>(h.cb.get(), h.cb.get(), n, h.partial.get(), h.counter.get(), s + S_BB, es_);
                    spmv_resid_norm(A, h.cx.get(), h.cb.get(), h.cr.get(),
                                    DotTarget{h.partial.get(), h.counter.get(), s + S_RR}, es_);
                }
                read_scalars();
                std::vector<Request*> started;
                for (Request* R : fresh) {
                    R->bn = std::sqrt(sc(R, S_BB));
                    if (R->bn == 0.0) {
                        MATAMG_HIP(hipMemsetAsync(R->h->cx.get(), 0, sizeof(double) * R->n, es_));
                        complete(R, AMG_OK);
                    } else if (std::sqrt(sc(R, S_RR)) / R->bn <= R->tol) {
                        R->rel_true = std::sqrt(sc(R, S_RR)) / R->bn;
                        complete(R, AMG_OK);
                    } else if (R->max_iter <= 0) {
                        complete(R, AMG_ERR_NOT_CONVERGED);
                    } else {
                        R->first = true;
                        R->cur = S_RZ0;
                        solving.push_back(R);
                    }
                }
                fresh.clear();
            }
            if (solving.empty()) continue;
            if (opt_.precision == AMG_PREC_FP32_HIER) run_step<float>(solving);
            else run_step<double>(solving);
            read_scalars();
            // convergence control of each request, as in the one-hierarchy solver
            std::vector<Request*> keep, confirm;
            for (Request* R : solving) {
                if (!R->first) R->cur = (R->cur == S_RZ0) ? S_RZ1 : S_RZ0;
                R->first = false;
                R->iters++;
                const double pq = sc(R, S_PQ), rzv = sc(R, R->cur);
                if (!(pq > 0.0) || !std::isfinite(pq) || !std::isfinite(rzv)) {
                    complete(R, AMG_ERR_BREAKDOWN);
                    continue;
                }
                const double rel = std::sqrt(sc(R, S_RR)) / R->bn;
                R->rel_true = rel;
                if (rel <= R->tol) {
                    confirm.push_back(R);
                } else if (R->iters >= R->max_iter) {
                    complete(R, AMG_ERR_NOT_CONVERGED);
                } else {
                    keep.push_back(R);
                }
            }
            if (!confirm.empty()) {
                for (Request* R : confirm) {
                    Hierarchy& h = *R->h;
                    double* s = sscal_.get() + (size_t)R->slot * S_NSCAL;
                    spmv_resid_norm(h.lev[0].A, h.cx.get(), h.cb.get(), h.cq.get(),
                                    DotTarget{h.partial.get(), h.counter.get(), s + S_TMP}, es_);
                }
                read_scalars();
                for (Request* R : confirm) {
                    R->rel_true = std::sqrt(sc(R, S_TMP)) / R->bn;
                    if (R->rel_true <= R->tol) {
                        complete(R, AMG_OK);
                        continue;
                    }
                    // residual replacement
                    Hierarchy& h = *R->h;
                    MATAMG_HIP(hipMemcpyAsync(h.cr.get(), h.cq.get(), sizeof(double) * R->n, hipMemcpyDeviceToDevice,
                                              es_));
                    if (R->iters >= R->max_iter) complete(R, AMG_ERR_NOT_CONVERGED);
                    else keep.push_back(R);
                }
            }
            // keep arrival order among the survivors
            std::sort(keep.begin(), keep.end(), [](const Request* a, const Request* b) { return a->id < b->id; });
            solving.swap(keep);
        } catch (const Error& e) {
            fail_all(fresh, e);
            fail_all(solving, e);
        }
    }
}

}  // namespace matamg
