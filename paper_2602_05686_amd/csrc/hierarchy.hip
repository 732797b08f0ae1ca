// Setup driver (sections 2 and 3 of the paper, per level: strength of
// connection, dropping, aggregation, prolongator smoothing, Galerkin
// product, auxiliary transfer; dense factorisation on the coarsest level),
// the V-cycle (Algorithm "Vcycle") and the outer preconditioned CG.
#include <chrono>
#include <cmath>
#include <cstdlib>

#include <exception>

#include "hierarchy.h"
#include "setup_kernels.h"

namespace matamg {

namespace {

uint64_t splitmix64_host(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
// one stream of draws per (purpose, level): aggregation priorities,
// prolongator power method, smoother power method
constexpr uint64_t kPurposeMis = 1, kPurposePf = 101, kPurposeCheb = 201;
uint64_t stream_key(uint64_t seed, uint64_t purpose, int level) {
    return splitmix64_host(seed + purpose + (uint64_t)level);
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Row blocks of A for the streaming kernels, computed on the device, and
// (if `pack`) the 16-bit packed columns.  MATAMG_CHECK_PARTITION=1 also runs
// the host walk and fails on any difference (used by the tests).
void make_blocks(DCsr& A, MemCounter* mc, hipStream_t s, bool pack = true, int cap = kStreamCap) {
    stream_partition(A, mc, s, pack, cap);
    const char* chk = std::getenv("MATAMG_CHECK_PARTITION");
    if (chk && chk[0] == '1') {
        std::vector<int> rp((size_t)A.n + 1);
        d2h(rp.data(), A.rowptr.get(), rp.size(), s);
        const int group = stream_group(rp.data(), A.n);
        std::vector<int> blk = stream_blocks(rp.data(), A.n, group, cap);
        std::vector<int> dev((size_t)A.nblk + 1);
        d2h(dev.data(), A.blk.get(), dev.size(), s);
        if (group != A.group || blk != dev)
            fail(AMG_ERR_HIP, "device row-block partition differs from the host walk (n=" + std::to_string(A.n) + ")");
    }
}

// Streaming blocks of up to kStreamCapWide entries for a large packed
// one-thread-per-row matrix: twice the bytes per workgroup, which the finest
// levels stream faster, while the setup kernels keep the kStreamCap blocks
// (sblk).  Kept only if the wider blocks pack too.
// MATAMG_WIDE_MIN_BLOCKS=<k> sets the block-count threshold of every level
// (used by the tests to run the wide kernels on small operators)
int wide_block_min(int level, bool fp32) {
    const char* e = std::getenv("MATAMG_WIDE_MIN_BLOCKS");
    if (e && e[0]) {
        const int v = std::atoi(e);
        if (v > 0) return v;
    }
    if (level == 0) return kWideBlockMinFine;
    return fp32 ? kWideBlockMinFp32 : kWideBlockMin;
}

void widen_stream_blocks(DCsr& A, int min_blocks, MemCounter* mc, hipStream_t s) {
    if (A.group != 1 || !A.col16 || A.cap != kStreamCap || A.nblk < min_blocks) return;
    DBuf<int> blk = std::move(A.blk), blkk = std::move(A.blkk), cbase = std::move(A.cbase),
              ustart = std::move(A.ustart);
    DBuf<uint16_t> col16 = std::move(A.col16), uoff = std::move(A.uoff);
    DBuf<uint32_t> urun = std::move(A.urun);
    const int nblk = A.nblk;
    const int64_t nuniq = A.nuniq;
    make_blocks(A, mc, s, true, kStreamCapWide);
    if (A.col16 && A.group == 1) {
        A.sblk = std::move(blk);
        A.snblk = nblk;
        return;
    }
    // not packable with wider blocks: back to the setup's partition
    A.blk = std::move(blk);
    A.blkk = std::move(blkk);
    A.cbase = std::move(cbase);
    A.col16 = std::move(col16);
    A.ustart = std::move(ustart);
    A.uoff = std::move(uoff);
    A.urun = std::move(urun);
    A.nuniq = nuniq;
    A.nblk = nblk;
    A.group = 1;
    A.cap = kStreamCap;
}

// reduction partials: one slot per block of the widest fused-reduction launch
void ensure_partial(Hierarchy& h, int nblocks) {
    const size_t need = (size_t)std::max(kMaxPartials, nblocks) + 1;
    if (h.partial.size() < need) h.partial.alloc(need, &h.mem);
}

int read_flag(int* dflag, hipStream_t s) {
    int v = 0;
    d2h(&v, dflag, 1, s);
    return v;
}

// lambda = ||dscale .* (A v)|| after `iters` normalised steps from a seeded start
double power_method(const DCsr& A, const double* dscale, int iters, uint64_t key, Hierarchy& h, hipStream_t s) {
    const int n = A.n;
    DBuf<double> v((size_t)n, &h.mem), w((size_t)n, &h.mem);
    fill_seeded_uniform(n, key, v.get(), s);
    dot<double>(v.get(), v.get(), n, h.partial.get(), h.counter.get(), h.scal.get() + S_TMP, s);
    scale_by_inv_norm(n, h.scal.get() + S_TMP, v.get(), v.get(), s);
    for (int it = 0; it < iters; ++it) {
        spmv_scale_norm(A, v.get(), dscale, w.get(), h.dt(S_TMP), s);
        if (it + 1 < iters) scale_by_inv_norm(n, h.scal.get() + S_TMP, w.get(), v.get(), s);
    }
    double nrm2 = 0.0;
    d2h(&nrm2, h.scal.get() + S_TMP, 1, s);
    return iters > 0 ? std::sqrt(nrm2) : 0.0;
}

void smoother_coefficients(Level& L, const amg_options& o) {
    L.c1.clear();
    L.c2.clear();
    if (o.smoother == AMG_SMOOTH_JACOBI || o.smoother == AMG_SMOOTH_JACOBI_SCALED) {
        // fixed weight, or jacobi_omega * 2 / beta with beta the Chebyshev
        // upper bound of the level's spectrum
        const double beta = o.cheb_boost * L.lam_cheb;
        const double w = (o.smoother == AMG_SMOOTH_JACOBI_SCALED && beta > 0.0) ? o.jacobi_omega * 2.0 / beta
                                                                                 : o.jacobi_omega;
        for (int k = 0; k < o.jacobi_sweeps; ++k) {
            L.c1.push_back(0.0);
            L.c2.push_back(w);
        }
        return;
    }
    const double beta = o.cheb_boost * L.lam_cheb;
    const double alpha = beta / o.cheb_ratio;
    const double theta = (beta + alpha) / 2.0, delta = (beta - alpha) / 2.0;
    const double s1 = theta / delta;
    double rho_old = 1.0 / s1;
    L.c1.push_back(0.0);
    L.c2.push_back(1.0 / theta);
    for (int k = 1; k < o.cheb_degree; ++k) {
        const double rho = 1.0 / (2.0 * s1 - rho_old);
        L.c1.push_back(rho * rho_old);
        L.c2.push_back(2.0 * rho / delta);
        rho_old = rho;
    }
}

template <typename T>
void alloc_work(Level& L, int n, bool coarse_only, MemCounter* mc);

template <>
void alloc_work<double>(Level& L, int n, bool coarse_only, MemCounter* mc) {
    L.b.alloc(n, mc);
    L.xa.alloc(n, mc);
    if (coarse_only) return;
    L.xb.alloc(n, mc);
    L.d.alloc(n, mc);
    L.r.alloc(n, mc);
}
template <>
void alloc_work<float>(Level& L, int n, bool coarse_only, MemCounter* mc) {
    L.fb.alloc(n, mc);
    L.fxa.alloc(n, mc);
    if (coarse_only) return;
    L.fxb.alloc(n, mc);
    L.fd.alloc(n, mc);
    L.fr.alloc(n, mc);
}

}  // namespace

// ------------------------------------------------------------------ V-cycle
template <typename T>
struct Vec;
template <>
struct Vec<double> {
    static double* b(Level& L) { return L.b.get(); }
    static double* xa(Level& L) { return L.xa.get(); }
    static double* xb(Level& L) { return L.xb.get(); }
    static double* d(Level& L) { return L.d.get(); }
    static double* r(Level& L) { return L.r.get(); }
    static const double* A(const DCsr& M) { return M.val.get(); }
    static const double* dinv(Level& L) { return L.dinv.get(); }
};
template <>
struct Vec<float> {
    static float* b(Level& L) { return L.fb.get(); }
    static float* xa(Level& L) { return L.fxa.get(); }
    static float* xb(Level& L) { return L.fxb.get(); }
    static float* d(Level& L) { return L.fd.get(); }
    static float* r(Level& L) { return L.fr.get(); }
    static const float* A(const DCsr& M) { return M.val32.get(); }
    static const float* dinv(Level& L) { return L.dinv32.get(); }
};

Hierarchy::~Hierarchy() {
    if (hscal) (void)hipHostFree(hscal);
    for (auto& g : graph)
        if (g) (void)hipGraphExecDestroy(g);
    if (ev_in) (void)hipEventDestroy(ev_in);
    give_stream(ws);  // back to the library's free list (its work stays ordered before later use)
}

// Steady-state duration of one smoother step on `level` (the fused
// Chebyshev SpMV that dominates the V-cycle): `reps` back-to-back launches
// between two events on the stream, on the level's own work vectors.
double Hierarchy::time_smoother(int level, int reps, hipStream_t s, double* bytes_per_launch) {
    Level& L = lev[level];
    const int n = L.A.n;
    hipEvent_t e0, e1;
    MATAMG_HIP(hipEventCreate(&e0));
    MATAMG_HIP(hipEventCreate(&e1));
    const double c1 = L.c1.size() > 1 ? L.c1[1] : 0.0, c2 = L.c2.size() > 1 ? L.c2[1] : L.c2[0];
    double ms_total = 0.0;
    auto run = [&](auto tag) {
        using T = decltype(tag);
        using V = Vec<T>;
        T* x = V::xa(L);
        T* y = V::xb(L);
        zero_async(V::b(L), sizeof(T) * n, s);
        zero_async(x, sizeof(T) * n, s);
        zero_async(V::d(L), sizeof(T) * n, s);
        spmv_smooth<T>(L.A, V::A(L.A), x, V::b(L), V::dinv(L), V::d(L), (T)c1, (T)c2, y, nullptr, nullptr,
                       DotTarget{}, s);
        MATAMG_HIP(hipEventRecord(e0, s));
        for (int k = 0; k < reps; ++k) {
            spmv_smooth<T>(L.A, V::A(L.A), x, V::b(L), V::dinv(L), V::d(L), (T)c1, (T)c2, y, nullptr, nullptr,
                           DotTarget{}, s);
            std::swap(x, y);
        }
        MATAMG_HIP(hipEventRecord(e1, s));
        MATAMG_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        MATAMG_HIP(hipEventElapsedTime(&ms, e0, e1));
        ms_total = ms;
    };
    if (fp32) run(float{});
    else run(double{});
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const double sz = fp32 ? 4.0 : 8.0;
    // val + col (as stored: 4 bytes, or 2 plus a base per block when packed)
    // + rowptr once, the gathered iterate once, b, D^{-1}, d read, d and x
    // written
    if (bytes_per_launch)
        *bytes_per_launch = (double)L.A.nnz * (sz + L.A.col_bytes()) + 4.0 * (L.A.n + 1) +
                            (L.A.col16 ? 4.0 * L.A.nblk : 0.0) + L.A.unique_bytes() + 6.0 * sz * L.A.n;
    return ms_total / reps;
}

// the solve's own stream, ordering event and pinned scalar mirror, created
// on the first solve (hierarchies driven by the solve server never need them)
void Hierarchy::ensure_solve_resources() {
    if (!hscal) MATAMG_HIP(hipHostMalloc((void**)&hscal, sizeof(double) * S_NSCAL, hipHostMallocDefault));
    if (!ws) ws = take_stream();
    if (!ev_in) MATAMG_HIP(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
}

// drop what only the parity getters read (strength values, drop masks,
// aggregates, coordinates and tensors); the V-cycle and CG do not use them
void Hierarchy::release_setup_data() {
    for (int l = 0; l < nlev; ++l) {
        Level& L = lev[l];
        L.S.release();
        L.mask.release();
        L.agg.release();
        L.x.release();
        L.sig.release();
        L.dir.release();
    }
}

DotTarget Hierarchy::dt(int slot) const { return DotTarget{partial.get(), counter.get(), scal.get() + slot}; }

namespace {

// filtered matrix of level l (the diagonal, lumped, and the entries its drop
// mask keeps, in the operator's stored order) with its 1-norm diagonal and
// that diagonal's inverse
void filtered_operator(Hierarchy& h, int l, DCsr& F, DBuf<double>& dt, DBuf<double>& dtinv, hipStream_t s) {
    Level& L = h.lev[l];
    MemCounter* mc = &h.mem;
    const int nl = L.A.n;
    F.n = F.m = nl;
    DBuf<int> cnt(nl, mc), tmp(scan_tmp_size(nl), mc);
    filter_count(L.A, L.mask.get(), cnt.get(), s);
    F.rowptr.alloc((size_t)nl + 1, mc);
    exclusive_scan(cnt.get(), F.rowptr.get(), nl, tmp.get(), s);
    int fnnz = 0;
    d2h(&fnnz, F.rowptr.get() + nl, 1, s);
    F.nnz = fnnz;
    F.col.alloc((size_t)(fnnz > 0 ? fnnz : 1), mc);
    F.val.alloc((size_t)(fnnz > 0 ? fnnz : 1), mc);
    dt.alloc(nl, mc);
    dtinv.alloc(nl, mc);
    filter_fill(L.A, L.mask.get(), L.dir.get(), F.rowptr.get(), F.col.get(), F.val.get(), dt.get(), dtinv.get(), s);
    make_blocks(F, mc, s, false);  // a few passes each: not worth packing
}

// damping and smoothed prolongator of level l from its filtered matrix F,
// F's 1-norm diagonal and the aggregates; sets lam_pf and omega
void smoothed_prolongator(Hierarchy& h, int l, const DCsr& F, const double* dt, const double* dtinv, DCsr& P,
                          hipStream_t s) {
    Level& L = h.lev[l];
    const amg_options& opt = h.opt;
    MemCounter* mc = &h.mem;
    const int nl = L.A.n;
    DBuf<int> cnt(nl, mc), tmp(scan_tmp_size(nl), mc);
    ensure_partial(h, std::max(stream_partials(F), stream_partials(L.A)));
    L.lam_pf = power_method(F, dtinv, opt.power_iters, stream_key(opt.seed, kPurposePf, l), h, s);
    L.omega = L.lam_pf > 0.0 ? opt.omega_sym / L.lam_pf : 0.0;
    DCsr Ph;
    Ph.n = nl;
    Ph.m = L.nc;
    phat_counts(nl, L.agg.get(), cnt.get(), s);
    Ph.rowptr.alloc((size_t)nl + 1, mc);
    exclusive_scan(cnt.get(), Ph.rowptr.get(), nl, tmp.get(), s);
    int pn = 0;
    d2h(&pn, Ph.rowptr.get() + nl, 1, s);
    Ph.nnz = pn;
    Ph.col.alloc((size_t)(pn > 0 ? pn : 1), mc);
    Ph.val.alloc((size_t)(pn > 0 ? pn : 1), mc);
    phat_fill(nl, L.agg.get(), Ph.rowptr.get(), Ph.col.get(), Ph.val.get(), s);
    spgemm(F, Ph, P, mc, s);
    prolongator_finalize(nl, P.rowptr.get(), P.col.get(), P.val.get(), L.agg.get(), dt, L.omega, s);
}

// Chebyshev bounds and coefficients of every smoothing level
void smoother_bounds(Hierarchy& h, hipStream_t s) {
    for (int k = 0; k + 1 < h.nlev; ++k) {
        Level& L = h.lev[k];
        L.lam_cheb = power_method(L.A, L.dinv.get(), h.opt.power_iters, stream_key(h.opt.seed, kPurposeCheb, k), h,
                                  s);
        smoother_coefficients(L, h.opt);
    }
}

// dense inverse of the coarsest operator through its Cholesky factor,
// enqueued on q (h.Ainv and work, nc * nc doubles each, allocated by the
// caller); *flag becomes 1 if the operator is not positive definite
void coarse_inverse_enqueue(Hierarchy& h, double* work, int* flag, hipStream_t q) {
    const Level& C = h.lev[h.nlev - 1];
    const int nc = C.A.n;
    zero_async(h.Ainv.get(), sizeof(double) * (size_t)nc * nc, q);
    densify(nc, C.A.rowptr.get(), C.A.col.get(), C.A.val.get(), h.Ainv.get(), q);
    dense_spd_inverse(nc, h.Ainv.get(), work, flag, q);
}

void coarse_inverse_alloc(Hierarchy& h) {
    const int nc = h.lev[h.nlev - 1].A.n;
    h.nL = nc;
    if (h.Ainv.size() != (size_t)nc * nc) h.Ainv.alloc((size_t)nc * nc, &h.mem);
}

void coarse_inverse_check(Hierarchy& h, int* flag, hipStream_t s) {
    if (read_flag(flag, s))
        fail(AMG_ERR_NOT_SPD, "coarsest operator is not positive definite (n=" + std::to_string(h.nL) + ")");
}

// A library stream that runs work beside stream s: everything enqueued on s
// before construction runs first, and join() makes s wait for all of it.
// Without a join (an error on s's side) the destructor waits for the side
// stream itself, so no buffer it uses is released to the pool while it runs.
class SideStream {
  public:
    explicit SideStream(hipStream_t s) : s_(s), side_(take_stream()) {
        if (hipEventCreateWithFlags(&ev_, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            give_stream(side_);
            fail(AMG_ERR_HIP, "hipEventCreateWithFlags failed");
        }
        if (hipEventRecord(ev_, s_) != hipSuccess || hipStreamWaitEvent(side_, ev_, 0) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipEventDestroy(ev_);
            give_stream(side_);
            fail(AMG_ERR_HIP, "ordering a side stream after the setup stream failed");
        }
    }
    SideStream(const SideStream&) = delete;
    SideStream& operator=(const SideStream&) = delete;
    hipStream_t get() const { return side_; }
    void join() {
        MATAMG_HIP(hipEventRecord(ev_, side_));
        MATAMG_HIP(hipStreamWaitEvent(s_, ev_, 0));
        joined_ = true;
    }
    ~SideStream() {
        if (!joined_) (void)hipStreamSynchronize(side_);
        (void)hipEventDestroy(ev_);
        give_stream(side_);
    }

  private:
    hipStream_t s_;
    hipStream_t side_;
    hipEvent_t ev_ = nullptr;
    bool joined_ = false;
};

// FP32 copies of A, D^{-1}, P and R on the smoothing levels
void cast_fp32(Hierarchy& h, hipStream_t s) {
    MemCounter* mc = &h.mem;
    for (int k = 0; k + 1 < h.nlev; ++k) {
        Level& L = h.lev[k];
        const int nl = L.A.n;
        if (!L.A.val32) L.A.val32.alloc((size_t)(L.A.nnz > 0 ? L.A.nnz : 1), mc);
        cast_vec<double, float>(L.A.nnz, L.A.val.get(), L.A.val32.get(), s);
        if (!L.dinv32) L.dinv32.alloc(nl, mc);
        cast_vec<double, float>(nl, L.dinv.get(), L.dinv32.get(), s);
        if (!L.P.val32) L.P.val32.alloc((size_t)(L.P.nnz > 0 ? L.P.nnz : 1), mc);
        cast_vec<double, float>(L.P.nnz, L.P.val.get(), L.P.val32.get(), s);
        if (!L.R.val32) L.R.val32.alloc((size_t)(L.R.nnz > 0 ? L.R.nnz : 1), mc);
        cast_vec<double, float>(L.R.nnz, L.R.val.get(), L.R.val32.get(), s);
    }
}

// a setup's or update's temporaries come from the pool in the order of its
// stream, unless the caller's thread already set a scope (the solve
// server's workers do)
//
// A scope opened here (not a server thread's) also keeps the temporaries it
// releases for its own later allocations on the stream; when it closes, the
// stream is synchronised and they become idle buffers, or, when it closes
// because of an error, they go back to the pool in stream order.
struct SetupAllocScope {
    bool own;  // declared first: initialised before the scope is opened
    AllocStreamScope scope;
    static hipStream_t pick(hipStream_t s) {
        if (!alloc_mode().pooled && pool_enabled()) {
            int dev = 0;
            MATAMG_HIP(hipGetDevice(&dev));
            keep_pool_memory(dev);
        }
        return alloc_mode().pooled ? alloc_mode().stream : s;
    }
    explicit SetupAllocScope(hipStream_t s)
        : own(!alloc_mode().pooled && pool_enabled()), scope(pick(s), alloc_mode().pooled || pool_enabled()) {
        if (own) alloc_mode().temps = true;
    }
    ~SetupAllocScope() {
        if (!own) return;
        const hipStream_t st = alloc_mode().stream;
        const bool clean = std::uncaught_exceptions() == 0 && hipStreamSynchronize(st) == hipSuccess;
        stream_cache_flush(st, clean);
    }
    SetupAllocScope(const SetupAllocScope&) = delete;
    SetupAllocScope& operator=(const SetupAllocScope&) = delete;
};

}  // namespace

std::unique_ptr<Hierarchy> build_hierarchy(int64_t n64, const int* rowptr, const int* col, const double* val,
                                           int64_t nelem, int npe, const int* elem_nodes,
                                           const double* elem_sigma, const double* coords,
                                           const amg_options& opt, bool host_ptrs, hipStream_t s,
                                           bool wide_blocks) {
    const double t0 = now_s();
    SetupAllocScope scope(s);
    auto hp = std::make_unique<Hierarchy>();
    Hierarchy& h = *hp;
    h.opt = opt;
    h.fp32 = opt.precision == AMG_PREC_FP32_HIER;
    const int n = (int)n64;
    const int dim = opt.dim;
    const int ncomp = dim * (dim + 1) / 2;
    MemCounter* mc = &h.mem;

    h.scal.alloc(S_NSCAL, mc);
    h.counter.alloc(1, mc);
    zero_async(h.counter.get(), sizeof(unsigned), s);
    zero_async(h.scal.get(), sizeof(double) * S_NSCAL, s);
    {
        // MATAMG_NO_GRAPH=1 runs every CG step eagerly (used to check the
        // captured graphs against direct launches)
        const char* ng = std::getenv("MATAMG_NO_GRAPH");
        h.use_graphs = !(ng && ng[0] == '1');
    }
    DBuf<int> flag(1, mc);
    zero_async(flag.get(), sizeof(int), s);

    // ---- level 1 inputs on the device
    Level& L0 = h.lev[0];
    int nnz = 0;
    if (host_ptrs) nnz = rowptr[n];
    else d2h(&nnz, rowptr + n, 1, s);
    if (nnz < 0) fail(AMG_ERR_INVALID_ARG, "rowptr[n] is negative");
    L0.A.n = L0.A.m = n;
    L0.A.nnz = nnz;
    L0.A.rowptr.alloc((size_t)n + 1, mc);
    L0.A.col.alloc((size_t)(nnz > 0 ? nnz : 1), mc);
    L0.A.val.alloc((size_t)(nnz > 0 ? nnz : 1), mc);
    L0.x.alloc((size_t)n * dim, mc);
    const hipMemcpyKind kind = host_ptrs ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    MATAMG_HIP(hipMemcpyAsync(L0.A.rowptr.get(), rowptr, sizeof(int) * ((size_t)n + 1), kind, s));
    MATAMG_HIP(hipMemcpyAsync(L0.A.col.get(), col, sizeof(int) * (size_t)nnz, kind, s));
    MATAMG_HIP(hipMemcpyAsync(L0.A.val.get(), val, sizeof(double) * (size_t)nnz, kind, s));
    MATAMG_HIP(hipMemcpyAsync(L0.x.get(), coords, sizeof(double) * (size_t)n * dim, kind, s));
    validate_csr(n, L0.A.rowptr.get(), L0.A.col.get(), nnz, flag.get(), s);
    if (read_flag(flag.get(), s)) fail(AMG_ERR_INVALID_ARG, "CSR columns unsorted, duplicated or out of range");
    check_finite(L0.A.val.get(), nnz, flag.get(), s);
    check_finite(L0.x.get(), (int64_t)n * dim, flag.get(), s);
    if (read_flag(flag.get(), s)) fail(AMG_ERR_INVALID_ARG, "a matrix value or a coordinate is not finite");

    // ---- Clement nodal tensors
    L0.sig.alloc((size_t)n * ncomp, mc);
    {
        DBuf<int> en;
        DBuf<double> es;
        const int* den = elem_nodes;
        const double* des = elem_sigma;
        if (host_ptrs && nelem > 0) {
            en.alloc((size_t)nelem * npe, mc);
            es.alloc((size_t)nelem * dim * dim, mc);
            MATAMG_HIP(hipMemcpyAsync(en.get(), elem_nodes, sizeof(int) * (size_t)nelem * npe, kind, s));
            MATAMG_HIP(hipMemcpyAsync(es.get(), elem_sigma, sizeof(double) * (size_t)nelem * dim * dim, kind, s));
            den = en.get();
            des = es.get();
        }
        check_finite(des, nelem * dim * dim, flag.get(), s);
        if (read_flag(flag.get(), s)) fail(AMG_ERR_INVALID_ARG, "an element tensor entry is not finite");
        Incidence inc;
        build_node_elements(den, nelem, npe, n, inc, flag.get(), mc, s);
        if (read_flag(flag.get(), s)) fail(AMG_ERR_INVALID_ARG, "element node id out of range");
        clement(n, dim, inc, des, L0.sig.get(), s);
        MATAMG_HIP(hipStreamSynchronize(s));
    }

    // ---- levels
    int l = 0;
    for (;; ++l) {
        Level& L = h.lev[l];
        const int nl = L.A.n;
        const int64_t nzl = L.A.nnz;
        L.dinv.alloc(nl, mc);
        make_blocks(L.A, mc, s);
        diag_inverse_blocks(L.A, L.dinv.get(), s);
        if (nl <= opt.max_coarse || l + 1 >= opt.max_levels) {
            if (nl > opt.max_coarse)
                fail(AMG_ERR_COARSENING_STAGNATED, "level cap reached with " + std::to_string(nl) + " unknowns");
            break;
        }
        // strength of connection and dropping
        L.dir.alloc(nl, mc);
        if (l == 0) detect_dirichlet(nl, L.A.rowptr.get(), L.A.col.get(), L.A.val.get(), L.dir.get(), s);
        else zero_async(L.dir.get(), nl, s);
        DBuf<double> minv;
        if (opt.soc == AMG_SOC_MATERIAL) {
            minv.alloc((size_t)nl * ncomp, mc);
            tensor_inverse(nl, dim, L.sig.get(), minv.get(), flag.get(), s);
            if (read_flag(flag.get(), s)) fail(AMG_ERR_NOT_SPD, "nodal tensor not SPD on level " + std::to_string(l));
        }
        DBuf<double> lval((size_t)(nzl > 0 ? nzl : 1), mc), ldiag(nl, mc);
        soc_values(L.A, dim, L.x.get(), minv.get(), L.dir.get(), opt.soc, lval.get(), ldiag.get(), s);
        L.S.alloc((size_t)(nzl > 0 ? nzl : 1), mc);
        L.mask.alloc((size_t)(nzl > 0 ? nzl : 1), mc);
        soc_mask(L.A, L.dir.get(), lval.get(), ldiag.get(), opt.theta, L.S.get(), L.mask.get(), s);
        if (opt.drop == AMG_DROP_CUT) {
            DBuf<uint8_t> keep((size_t)(nzl > 0 ? nzl : 1), mc);
            cut_drop(L.A, L.dir.get(), lval.get(), ldiag.get(), opt.theta, keep.get(), L.mask.get(), s);
        }
        lval.release();
        ldiag.release();
        minv.release();

        // the filtered matrix holds the diagonal and exactly the kept entries
        // in stored order, so the independent set and the aggregation walk
        // its pattern with no mask, and the prolongator smooths with it
        DCsr F;
        DBuf<double> dt, dtinv;
        filtered_operator(h, l, F, dt, dtinv, s);

        // distance-2 maximal independent set, synchronous rounds
        {
            DBuf<uint8_t> state(nl, mc);
            DBuf<uint64_t> t1(nl, mc), t2(nl, mc);
            // rounds run in batches with one read-back per batch: a round
            // after the last undecided node is gone changes nothing, and the
            // per-round undecided counts give the exact round count
            constexpr int kMisBatch = 4;
            DBuf<int> und(kMisBatch, mc);
            const uint64_t key = stream_key(opt.seed, kPurposeMis, l);
            mis_init(nl, L.dir.get(), state.get(), s);
            int rounds = 0;
            for (bool done = false; !done;) {
                zero_async(und.get(), sizeof(int) * kMisBatch, s);
                for (int j = 0; j < kMisBatch; ++j)
                    mis_round(F, nullptr, key, state.get(), t1.get(), t2.get(), und.get() + j, s);
                int left[kMisBatch];
                d2h(left, und.get(), kMisBatch, s);
                for (int j = 0; j < kMisBatch && !done; ++j) {
                    ++rounds;
                    done = left[j] == 0;
                }
                if (!done && rounds > nl + 1) fail(AMG_ERR_HIP, "distance-2 MIS did not terminate");
            }
            L.mis_rounds = rounds;
            t1.release();
            t2.release();
            DBuf<int> flags(nl, mc), rank((size_t)nl + 1, mc), tmp(scan_tmp_size(nl), mc), phase2(nl, mc);
            agg_root_flags(nl, state.get(), flags.get(), s);
            exclusive_scan(flags.get(), rank.get(), nl, tmp.get(), s);
            int nagg = 0;
            d2h(&nagg, rank.get() + nl, 1, s);
            if (nagg <= 0 || nagg >= nl)
                fail(AMG_ERR_COARSENING_STAGNATED,
                     "aggregation did not reduce level " + std::to_string(l) + " (" + std::to_string(nagg) + " of " +
                         std::to_string(nl) + ")");
            L.nc = nagg;
            L.agg.alloc(nl, mc);
            agg_assign(nl, F.rowptr.get(), F.col.get(), nullptr, L.dir.get(), state.get(), rank.get(), phase2.get(),
                       L.agg.get(), flags.get(), und.get(), s);
        }

        smoothed_prolongator(h, l, F, dt.get(), dtinv.get(), L.P, s);
        F = DCsr();
        dt.release();
        dtinv.release();
        transpose(L.P, L.R, mc, s);
        Level& C = h.lev[l + 1];
        {
            DCsr AP;
            spgemm(L.A, L.P, AP, mc, s);
            spgemm(L.R, AP, C.A, mc, s);
        }
        C.A.n = C.A.m = L.nc;
        // coarse coordinates and tensors: aggregate means
        C.x.alloc((size_t)L.nc * dim, mc);
        C.sig.alloc((size_t)L.nc * ncomp, mc);
        {
            Incidence mem;
            build_aggregate_members(L.agg.get(), nl, L.nc, mem, mc, s);
            coarse_aux(L.nc, dim, mem, L.x.get(), L.sig.get(), C.x.get(), C.sig.get(), s);
            MATAMG_HIP(hipStreamSynchronize(s));
        }
        h.nlev = l + 2;
    }
    h.nlev = l + 1;
    ensure_partial(h, stream_partials(h.lev[0].A));

    {
        // the dense coarse inverse reads only the coarsest operator and runs
        // a few workgroups at a time: it goes on a second stream while the
        // transfer operators are partitioned, the operators' partitions
        // widened and the smoother bounds estimated on this one
        coarse_inverse_alloc(h);
        DBuf<double> work((size_t)h.nL * h.nL, mc);
        DBuf<int> cflag(1, mc);
        SideStream side(s);
        coarse_inverse_enqueue(h, work.get(), cflag.get(), side.get());
        // the transfer operators' streaming partitions serve only the
        // V-cycle, so they are made here, beside the coarse inverse too
        for (int k = 0; k + 1 < h.nlev; ++k) {
            make_blocks(h.lev[k].P, mc, s);
            make_blocks(h.lev[k].R, mc, s);
        }
        if (wide_blocks)
            for (int k = 0; k < h.nlev; ++k) widen_stream_blocks(h.lev[k].A, wide_block_min(k, h.fp32), mc, s);
        smoother_bounds(h, s);
        side.join();
        coarse_inverse_check(h, cflag.get(), s);
    }

    // work vectors and reduced-precision copies
    for (int k = 0; k < h.nlev; ++k) {
        Level& L = h.lev[k];
        const int nl = L.A.n;
        const bool coarsest = (k == h.nlev - 1);
        alloc_work<double>(L, nl, coarsest, mc);
        if (h.fp32) alloc_work<float>(L, nl, coarsest, mc);
    }
    if (h.fp32) cast_fp32(h, s);
    const size_t n0 = (size_t)h.lev[0].A.n;
    h.cx.alloc(n0, mc);
    h.cr.alloc(n0, mc);
    h.cz.alloc(n0, mc);
    h.cp.alloc(n0, mc);
    h.cq.alloc(n0, mc);
    MATAMG_HIP(hipStreamSynchronize(s));
    h.t_setup = now_s() - t0;
    return hp;
}

// New values of A on the setup's pattern: the value-dependent steps run again
// on the kept masks, aggregates, coordinates and tensors (every pattern stays
// as it is, so the new values are written into the existing arrays).
void update_values(Hierarchy& h, const double* val, bool host_ptrs, hipStream_t s) {
    const double t0 = now_s();
    SetupAllocScope scope(s);
    MemCounter* mc = &h.mem;
    Level& L0 = h.lev[0];
    const int n = L0.A.n;
    for (int l = 0; l + 1 < h.nlev; ++l)
        if (!h.lev[l].mask || !h.lev[l].agg || !h.lev[l].dir)
            fail(AMG_ERR_INVALID_ARG, "the hierarchy no longer holds the masks and aggregates an update reuses");
    DBuf<int> flag(1, mc);
    zero_async(flag.get(), sizeof(int), s);
    {
        // checked before anything of the hierarchy changes
        const size_t nnz = (size_t)L0.A.nnz;
        DBuf<double> v(nnz > 0 ? nnz : 1, mc);
        MATAMG_HIP(hipMemcpyAsync(v.get(), val, sizeof(double) * nnz,
                                  host_ptrs ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
        check_finite(v.get(), (int64_t)nnz, flag.get(), s);
        if (read_flag(flag.get(), s)) fail(AMG_ERR_INVALID_ARG, "a new matrix value is not finite");
        if (h.nlev > 1) {
            DBuf<uint8_t> dir(n > 0 ? n : 1, mc);
            detect_dirichlet(n, L0.A.rowptr.get(), L0.A.col.get(), v.get(), dir.get(), s);
            bytes_differ(n, dir.get(), L0.dir.get(), flag.get(), s);
            if (read_flag(flag.get(), s))
                fail(AMG_ERR_INVALID_ARG, "the Dirichlet rows of the new values differ from the setup's");
        }
        MATAMG_HIP(hipMemcpyAsync(L0.A.val.get(), v.get(), sizeof(double) * nnz, hipMemcpyDeviceToDevice, s));
    }
    auto take_values = [&](DCsr& dst, const DCsr& src, const char* what) {
        if (src.nnz != dst.nnz || src.n != dst.n)
            fail(AMG_ERR_HIP, std::string("the pattern of ") + what + " changed in an update");
        MATAMG_HIP(hipMemcpyAsync(dst.val.get(), src.val.get(), sizeof(double) * (size_t)dst.nnz,
                                  hipMemcpyDeviceToDevice, s));
    };
    for (int l = 0; l < h.nlev; ++l) {
        Level& L = h.lev[l];
        diag_inverse_blocks(L.A, L.dinv.get(), s);
        if (l + 1 == h.nlev) break;
        {
            DCsr F, P;
            DBuf<double> dt, dtinv;
            filtered_operator(h, l, F, dt, dtinv, s);
            smoothed_prolongator(h, l, F, dt.get(), dtinv.get(), P, s);
            take_values(L.P, P, "P");
        }
        {
            DCsr R;
            transpose(L.P, R, mc, s);
            take_values(L.R, R, "R");
        }
        DCsr AP, Ac;
        spgemm(L.A, L.P, AP, mc, s);
        spgemm(L.R, AP, Ac, mc, s);
        take_values(h.lev[l + 1].A, Ac, "a coarse operator");
    }
    {
        // as in the setup: the dense coarse inverse beside the smoother bounds
        coarse_inverse_alloc(h);
        DBuf<double> work((size_t)h.nL * h.nL, mc);
        DBuf<int> cflag(1, mc);
        SideStream side(s);
        coarse_inverse_enqueue(h, work.get(), cflag.get(), side.get());
        smoother_bounds(h, s);
        side.join();
        coarse_inverse_check(h, cflag.get(), s);
    }
    if (h.fp32) cast_fp32(h, s);
    // the captured CG steps hold the old smoother coefficients as kernel arguments
    for (auto& g : h.graph)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    MATAMG_HIP(hipStreamSynchronize(s));
    h.t_update = now_s() - t0;
}

template <typename T>
void Hierarchy::vcycle_t(const double* r64, double* z64, DotTarget rz, hipStream_t s) {
    using V = Vec<T>;
    const int L = nlev;
    if (L == 1) {
        dense_gemv<double>(nL, Ainv.get(), r64, z64, s);
        dot<double>(r64, z64, nL, rz.partial, rz.counter, rz.result, s);
        return;
    }
    T* cur[16];
    // restriction sweep
    for (int l = 0; l + 1 < L; ++l) {
        Level& Lv = lev[l];
        const int n = Lv.A.n;
        T* b;
        const double* b64 = nullptr;
        if constexpr (std::is_same<T, double>::value) {
            b = (l == 0) ? const_cast<double*>(r64) : V::b(Lv);
        } else {
            b = V::b(Lv);
            if (l == 0) b64 = r64;
        }
        T* x = V::xa(Lv);
        T* y = V::xb(Lv);
        // the first step from zero; below the finest level the restriction
        // that made b has already taken it
        if (l == 0) smooth_first<T>(n, b64, b, V::dinv(Lv), (T)Lv.c2[0], V::d(Lv), x, s);
        for (size_t k = 1; k < Lv.c1.size(); ++k) {
            spmv_smooth<T>(Lv.A, V::A(Lv.A), x, b, V::dinv(Lv), V::d(Lv), (T)Lv.c1[k], (T)Lv.c2[k], y, nullptr,
                           nullptr, DotTarget{}, s);
            std::swap(x, y);
        }
        cur[l] = x;
        spmv_resid<T>(Lv.A, V::A(Lv.A), x, b, V::r(Lv), s);
        Level& Ln = lev[l + 1];
        if (l + 2 < L)
            spmv_restrict_first<T>(Lv.R, V::A(Lv.R), V::r(Lv), V::b(Ln), V::dinv(Ln), (T)Ln.c2[0], V::d(Ln),
                                   V::xa(Ln), s);
        else
            spmv<T>(Lv.R, V::A(Lv.R), V::r(Lv), V::b(Ln), s);
    }
    // coarsest level
    Level& Lc = lev[L - 1];
    dense_gemv<T>(nL, Ainv.get(), V::b(Lc), V::xa(Lc), s);
    cur[L - 1] = V::xa(Lc);
    // prolongation sweep
    for (int l = L - 2; l >= 0; --l) {
        Level& Lv = lev[l];
        T* b;
        if constexpr (std::is_same<T, double>::value) b = (l == 0) ? const_cast<double*>(r64) : V::b(Lv);
        else b = V::b(Lv);
        T* x = cur[l];
        T* y = (x == V::xa(Lv)) ? V::xb(Lv) : V::xa(Lv);
        spmv_add<T>(Lv.P, V::A(Lv.P), cur[l + 1], x, x, s);
        const size_t steps = Lv.c1.size();
        for (size_t k = 0; k < steps; ++k) {
            const bool last = (l == 0 && k + 1 == steps);
            T* out = y;
            double* out64 = nullptr;
            if (last) {
                if constexpr (std::is_same<T, double>::value) out = z64;
                else out64 = z64;
            }
            const double* dv = last ? r64 : nullptr;
            spmv_smooth<T>(Lv.A, V::A(Lv.A), x, b, V::dinv(Lv), V::d(Lv), (T)(k == 0 ? 0.0 : Lv.c1[k]), (T)Lv.c2[k],
                           out, out64, dv, last ? rz : DotTarget{}, s);
            if (!last) std::swap(x, y);
        }
        cur[l] = x;
    }
}

void Hierarchy::vcycle(const double* r, double* z, DotTarget rz, hipStream_t s) {
    if (fp32) vcycle_t<float>(r, z, rz, s);
    else vcycle_t<double>(r, z, rz, s);
}

// Algorithmic HBM bytes of one V-cycle in the implemented kernel schedule:
// every streaming SpMV reads val, col and rowptr once and each listed vector
// once; the coarse GEMV reads the dense inverse.
double Hierarchy::vcycle_alg_bytes() const {
    const double s = fp32 ? 4.0 : 8.0;
    double bytes = 0.0;
    for (int l = 0; l + 1 < nlev; ++l) {
        const Level& L = lev[l];
        const double n = L.A.n, nc = L.nc;
        const double steps = (double)L.c1.size();
        // a matrix: values, columns as stored for the streaming kernels (4
        // bytes, or 2 when packed, plus one base per row block), row pointer
        auto matrix = [&](const DCsr& M) {
            return (double)M.nnz * (s + M.col_bytes()) + 4.0 * (M.n + 1) + (M.col16 ? 4.0 * M.nblk : 0.0) +
                   M.unique_bytes();
        };
        // smoother SpMVs: (steps-1) pre + steps post; one residual SpMV
        const double n_spmv = (steps - 1.0) + steps + 1.0;
        bytes += n_spmv * matrix(L.A);
        bytes += matrix(L.R);  // R r
        bytes += matrix(L.P);  // x += P e
        // vectors: the finest level's first step reads b, dinv, writes d, x
        // (4); each smoother SpMV reads x, b, dinv, d and writes d, x (6);
        // residual reads x, b, writes r (3); restriction reads r, writes b_c
        // and, above the coarsest level, takes that level's first step
        // (reads dinv_c, writes d_c, x_c); prolongation reads e_c, x, writes x
        const double vec_n = (l == 0 ? 4.0 : 0.0) + 6.0 * ((steps - 1.0) + steps) + 3.0 + 1.0 + 2.0;
        const double vec_c = 1.0 + 1.0 + (l + 2 < nlev ? 3.0 : 0.0);
        bytes += vec_n * s * n + vec_c * s * nc;
    }
    bytes += 8.0 * (double)nL * nL + 2.0 * s * nL;
    return bytes;
}

// ---------------------------------------------------------------------- PCG
// One captured graph per parity of the iteration counter: the V-cycle and
// search-direction update of step k followed by q = A p and the x / r update
// of step k + 1.  All operands are hierarchy-owned buffers, so the two
// graphs are captured once per hierarchy and replayed every step; the
// convergence test reads the device scalars after each replay.
hipGraphExec_t Hierarchy::step_graph(int cur) {
    const int g = (cur == S_RZ0) ? 0 : 1;
    if (graph[g]) return graph[g];
    const int nxt = (cur == S_RZ0) ? S_RZ1 : S_RZ0;
    const DCsr& A = lev[0].A;
    const int n = A.n;
    MATAMG_HIP(hipStreamBeginCapture(ws, hipStreamCaptureModeThreadLocal));
    vcycle(cr.get(), cz.get(), dt(nxt), ws);
    cg_direction(n, cp.get(), cz.get(), scal.get() + nxt, scal.get() + cur, ws);
    spmv_dot(A, cp.get(), cq.get(), dt(S_PQ), ws);
    cg_update(n, cx.get(), cr.get(), cp.get(), cq.get(), scal.get() + nxt, scal.get() + S_PQ, dt(S_RR), ws);
    hipGraph_t gr = nullptr;
    MATAMG_HIP(hipStreamEndCapture(ws, &gr));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    MATAMG_HIP(e);
    graph[g] = ex;
    return ex;
}

// the widest fused reduction of a solve: the finest operator's streaming
// launches (q = A p, residual norms, the last smoothing step's r.z) and the
// vector kernels' grids
size_t pcg_partials(const Hierarchy& h) {
    return (size_t)std::max(kMaxPartials, stream_partials(h.lev[0].A)) + 1;
}

// The PCG iteration on an explicit workspace (see PcgWork): the convergence
// test reads the device scalars after every step through w.hscal.
amg_status pcg_run(Hierarchy& h, const PcgWork& w, const double* b, double tol, int max_iter, int* iters_out,
                   double* rel_out) {
    const DCsr& A = h.lev[0].A;
    const int n = A.n;
    hipStream_t ws = w.stream;
    double* x = w.x;
    double* r = w.r;
    double* z = w.z;
    double* p = w.p;
    double* q = w.q;
    auto dt = [&](int slot) { return DotTarget{w.partial, w.counter, w.scal + slot}; };
    auto read_scal = [&]() {
        MATAMG_HIP(hipMemcpyAsync(w.hscal, w.scal, sizeof(double) * S_NSCAL, hipMemcpyDeviceToHost, ws));
        MATAMG_HIP(hipStreamSynchronize(ws));
    };
    amg_status st = AMG_ERR_NOT_CONVERGED;
    int iters = 0;
    double rel_true = 0.0;
    dot<double>(b, b, n, w.partial, w.counter, w.scal + S_BB, ws);
    spmv_resid_norm(A, x, b, r, dt(S_RR), ws);
    read_scal();
    if (!std::isfinite(w.hscal[S_BB]))
        fail(AMG_ERR_INVALID_ARG, "the right-hand side is not finite (or its 2-norm overflows)");
    if (!std::isfinite(w.hscal[S_RR])) fail(AMG_ERR_INVALID_ARG, "the initial guess is not finite");
    const double bn = std::sqrt(w.hscal[S_BB]);
    if (bn == 0.0) {
        zero_async(x, sizeof(double) * n, ws);
        st = AMG_OK;
    } else if (std::sqrt(w.hscal[S_RR]) / bn <= tol) {
        rel_true = std::sqrt(w.hscal[S_RR]) / bn;
        st = AMG_OK;
    } else if (max_iter > 0) {
        // first step eagerly: z = M r, p = z, q = A p, x and r updated
        int cur = S_RZ0;
        h.vcycle(r, z, dt(cur), ws);
        cg_direction(n, p, z, w.scal + cur, nullptr, ws);
        spmv_dot(A, p, q, dt(S_PQ), ws);
        cg_update(n, x, r, p, q, w.scal + cur, w.scal + S_PQ, dt(S_RR), ws);
        for (int it = 1;; ++it) {
            read_scal();
            iters = it;
            const double pq = w.hscal[S_PQ], rzv = w.hscal[cur];
            if (!(pq > 0.0) || !std::isfinite(pq) || !std::isfinite(rzv)) {
                st = AMG_ERR_BREAKDOWN;
                break;
            }
            const double rel = std::sqrt(w.hscal[S_RR]) / bn;
            rel_true = rel;
            if (rel <= tol) {
                spmv_resid_norm(A, x, b, q, dt(S_TMP), ws);
                read_scal();
                rel_true = std::sqrt(w.hscal[S_TMP]) / bn;
                if (rel_true <= tol) {
                    st = AMG_OK;
                    break;
                }
                // residual replacement
                MATAMG_HIP(hipMemcpyAsync(r, q, sizeof(double) * n, hipMemcpyDeviceToDevice, ws));
            }
            if (it >= max_iter) break;
            const int nxt = (cur == S_RZ0) ? S_RZ1 : S_RZ0;
            if (w.graphs) {
                MATAMG_HIP(hipGraphLaunch(h.step_graph(cur), ws));
            } else {
                h.vcycle(r, z, dt(nxt), ws);
                cg_direction(n, p, z, w.scal + nxt, w.scal + cur, ws);
                spmv_dot(A, p, q, dt(S_PQ), ws);
                cg_update(n, x, r, p, q, w.scal + nxt, w.scal + S_PQ, dt(S_RR), ws);
            }
            cur = nxt;
        }
    }
    *iters_out = iters;
    *rel_out = rel_true;
    return st;
}

amg_status pcg_solve(Hierarchy& h, const double* b_in, double* x_io, double tol, int max_iter, bool host_ptrs,
                     hipStream_t s, amg_solve_info* info) {
    const double t0 = now_s();
    const int n = h.lev[0].A.n;
    h.ensure_solve_resources();
    hipStream_t ws = h.ws;
    // order after the caller's earlier work on its stream
    MATAMG_HIP(hipEventRecord(h.ev_in, s));
    MATAMG_HIP(hipStreamWaitEvent(ws, h.ev_in, 0));
    const double* b = b_in;
    double* x = h.cx.get();
    if (host_ptrs) {
        if (!h.cb) h.cb.alloc(n, &h.mem);
        h2d(h.cb.get(), b_in, n, ws);
        b = h.cb.get();
        h2d(x, x_io, n, ws);
    } else {
        MATAMG_HIP(hipMemcpyAsync(x, x_io, sizeof(double) * n, hipMemcpyDeviceToDevice, ws));
    }
    // the captured step graphs hold these buffers
    PcgWork w{x, h.cr.get(), h.cz.get(), h.cp.get(), h.cq.get(), h.scal.get(), h.partial.get(), h.counter.get(),
              h.hscal, ws, h.use_graphs};
    int iters = 0;
    double rel_true = 0.0;
    const amg_status st = pcg_run(h, w, b, tol, max_iter, &iters, &rel_true);
    if (host_ptrs) d2h(x_io, x, n, ws);
    else MATAMG_HIP(hipMemcpyAsync(x_io, x, sizeof(double) * n, hipMemcpyDeviceToDevice, ws));
    MATAMG_HIP(hipStreamSynchronize(ws));
    if (info) {
        info->iterations = iters;
        info->rel_res_true = rel_true;
        info->t_solve_s = now_s() - t0;
        info->status = st;
    }
    return st;
}

}  // namespace matamg
