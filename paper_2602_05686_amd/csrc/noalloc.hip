// The allocation-free PCG solve: amg_pcg_solve's iteration with its
// workspace (the CG vectors r, z, p, q, the device scalars and the reduction
// partials) in one file-scope device array instead of hierarchy buffers, on
// the caller's stream, without captured graphs, solve stream, event or
// pinned mirror, so that the call allocates nothing.
#include <chrono>
#include <mutex>

#include "hierarchy.h"

namespace matamg {
namespace {

// 256 MiB of workspace on every device the library runs on, held until the
// process ends.  Host code never passes `scratch` itself to a kernel (in host
// code the name stands for a host-side shadow); it uses the device address
// that hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = 256ull << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// device address of `scratch` on the current device, looked up once per device
double* scratch_on_current_device() {
    int dev = 0;
    MATAMG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(AMG_ERR_HIP, "device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        MATAMG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) fail(AMG_ERR_HIP, "hipGetSymbolAddress returned a null address for the solve workspace");
        g_scratch[dev] = static_cast<double*>(ptr);
    }
    return g_scratch[dev];
}

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

// bytes of workspace a solve on h needs: four vectors, the scalars, the
// partials and the counter, each piece 256-byte aligned
size_t noalloc_need_bytes(const Hierarchy& h) {
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t n = (size_t)h.lev[0].A.n;
    return 4 * up(n * sizeof(double)) + up(S_NSCAL * sizeof(double)) + up(pcg_partials(h) * sizeof(double)) +
           up(sizeof(unsigned));
}

amg_status pcg_solve_noalloc(Hierarchy& h, const double* b, double* x, double tol, int max_iter, hipStream_t s,
                             amg_solve_info* info) {
    const auto t0 = std::chrono::steady_clock::now();
    const size_t need = noalloc_need_bytes(h);
    if (need > kScratchBytes)
        fail(AMG_ERR_INVALID_ARG, "the allocation-free solve needs " + std::to_string(need) + " bytes of workspace for " +
                                      std::to_string(h.lev[0].A.n) + " unknowns; it has " +
                                      std::to_string(kScratchBytes));
    double* base = scratch_on_current_device();
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t n = (size_t)h.lev[0].A.n;
    char* cur = reinterpret_cast<char*>(base);
    auto take = [&](size_t bytes) {
        char* p = cur;
        cur += up(bytes);
        return p;
    };
    double* r = reinterpret_cast<double*>(take(n * sizeof(double)));
    double* z = reinterpret_cast<double*>(take(n * sizeof(double)));
    double* p = reinterpret_cast<double*>(take(n * sizeof(double)));
    double* q = reinterpret_cast<double*>(take(n * sizeof(double)));
    double* scal = reinterpret_cast<double*>(take(S_NSCAL * sizeof(double)));
    double* partial = reinterpret_cast<double*>(take(pcg_partials(h) * sizeof(double)));
    unsigned* counter = reinterpret_cast<unsigned*>(take(sizeof(unsigned)));
    // the workspace keeps the previous call's contents: clear what the
    // reductions read before they write it
    zero_async(scal, sizeof(double) * S_NSCAL, s);
    zero_async(counter, sizeof(unsigned), s);
    double hscal[S_NSCAL] = {};
    PcgWork w{x, r, z, p, q, scal, partial, counter, hscal, s, false};
    int iters = 0;
    double rel_true = 0.0;
    const amg_status st = pcg_run(h, w, b, tol, max_iter, &iters, &rel_true);
    MATAMG_HIP(hipStreamSynchronize(s));
    if (info) {
        info->iterations = iters;
        info->rel_res_true = rel_true;
        info->t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        info->status = st;
    }
    return st;
}

}  // namespace matamg
