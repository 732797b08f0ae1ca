// Internal definitions shared by the HIP sources of the library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "../../include/amg.h"

namespace matamg {

// ---------------------------------------------------------------------------
// errors: thrown inside the library, converted to amg_status at the boundary
// ---------------------------------------------------------------------------
struct Error {
    amg_status code;
    std::string msg;
};

[[noreturn]] void fail(amg_status code, const std::string& msg);

// A failed call is reported once: the runtime's last-error value it leaves
// behind is cleared, so that it cannot resurface in a later, unrelated call.
#define MATAMG_HIP(call)                                                                        \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) {                                                                 \
            (void)hipGetLastError();                                                            \
            ::matamg::fail(e_ == hipErrorOutOfMemory ? AMG_ERR_OUT_OF_MEMORY : AMG_ERR_HIP,     \
                           std::string(#call) + ": " + hipGetErrorString(e_));                  \
        }                                                                                       \
    } while (0)

#define MATAMG_LAUNCH_CHECK() MATAMG_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
struct MemCounter {
    int64_t bytes = 0;
    int64_t peak = 0;
    void add(int64_t b) {
        bytes += b;
        if (bytes > peak) peak = bytes;
    }
};

// Stream-ordered allocation.  Code that builds hierarchies (setup, the solve
// server's threads) sets a per-thread stream; device buffers created and
// released under it come from the device's memory pool (hipMallocAsync /
// hipFreeAsync on that stream) instead of hipMalloc / hipFree, whose release
// waits for every stream of the device and whose mapping of fresh memory is
// slow.
struct AllocMode {
    bool pooled = false;
    hipStream_t stream = nullptr;
    bool idle = false;   // released buffers are idle (the device is synchronised): keep them for reuse
    bool temps = false;  // released buffers are kept for later allocations on the same stream
};
AllocMode& alloc_mode();
struct AllocStreamScope {
    AllocMode prev;
    explicit AllocStreamScope(hipStream_t s, bool pooled = true) : prev(alloc_mode()) {
        alloc_mode() = AllocMode{pooled, s};
    }
    ~AllocStreamScope() { alloc_mode() = prev; }
    AllocStreamScope(const AllocStreamScope&) = delete;
    AllocStreamScope& operator=(const AllocStreamScope&) = delete;
};
// Idle device buffers kept for reuse.  A stream-ordered allocation or free
// costs 0.1-0.25 ms of host time each in this runtime (a hierarchy holds
// a few hundred buffers), so the buffers of a freed hierarchy, released once
// the device is idle, are kept here by device and exact byte size and handed
// to the next pooled allocation of that size on the device, whatever its
// stream.  At most kIdleCacheBytes per process are kept.
constexpr uint64_t kIdleCacheBytes = 32ull << 30;
void* idle_take(size_t bytes);            // nullptr if none is kept
bool idle_put(void* p, size_t bytes);     // false when the cache is full
// frees the idle buffers of the current device on stream s; returns their bytes
uint64_t idle_trim(hipStream_t s);
// Buffers released in stream order during a setup, kept (by stream and exact
// size) for the setup's later allocations on the same stream, which are
// ordered after every use of the buffer; at the setup's end they become idle
// buffers (the stream synchronised) or, after a failure, go back to the pool.
void* stream_take(hipStream_t s, size_t bytes);
bool stream_put(hipStream_t s, void* p, size_t bytes);
void stream_cache_flush(hipStream_t s, bool to_idle);
// a per-device solve stream from the library's free list (created when the
// list is empty; default priority), and its return
hipStream_t take_stream();
void give_stream(hipStream_t s);
// keep memory freed to the device's default pool for reuse (idempotent)
void keep_pool_memory(int device);
// false when MATAMG_NO_POOL=1 asks for plain hipMalloc / hipFree everywhere
bool pool_enabled();
// a per-device stream of the library (default priority, created once) on which
// the pooled buffers of a freed hierarchy are handed back
hipStream_t release_stream();

template <typename T>
class DBuf {
  public:
    DBuf() = default;
    DBuf(size_t n, MemCounter* mc = nullptr) { alloc(n, mc); }
    ~DBuf() { release(); }
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept { swap(o); }
    DBuf& operator=(DBuf&& o) noexcept {
        if (this != &o) {
            release();
            swap(o);
        }
        return *this;
    }
    void alloc(size_t n, MemCounter* mc = nullptr) {
        release();
        n_ = n;
        mc_ = mc;
        if (n == 0) return;
        const AllocMode m = alloc_mode();
        pooled_ = m.pooled;
        hipError_t e = hipSuccess;
        if (pooled_) {
            p_ = m.temps ? static_cast<T*>(stream_take(m.stream, n * sizeof(T))) : nullptr;
            if (!p_) p_ = static_cast<T*>(idle_take(n * sizeof(T)));
            if (!p_) e = hipMallocAsync((void**)&p_, n * sizeof(T), m.stream);
        } else {
            e = hipMalloc(&p_, n * sizeof(T));
        }
        if (e != hipSuccess) {
            p_ = nullptr;
            n_ = 0;
            fail(AMG_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
        }
        if (mc_) mc_->add((int64_t)(n * sizeof(T)));
    }
    void release() {
        if (p_) {
            // a pooled buffer goes back to the pool in the order of the current
            // thread's stream (the null stream outside a scope: callers free
            // hierarchies only once the device is idle)
            if (pooled_) {
                const AllocMode& m = alloc_mode();
                const size_t b = n_ * sizeof(T);
                const bool kept = (m.idle && idle_put(p_, b)) || (m.temps && stream_put(m.stream, p_, b));
                if (!kept) (void)hipFreeAsync(p_, m.stream);
            } else {
                (void)hipFree(p_);
            }
            if (mc_) mc_->add(-(int64_t)(n_ * sizeof(T)));
        }
        p_ = nullptr;
        n_ = 0;
    }
    T* get() const { return p_; }
    size_t size() const { return n_; }
    explicit operator bool() const { return p_ != nullptr; }

  private:
    void swap(DBuf& o) {
        std::swap(p_, o.p_);
        std::swap(n_, o.n_);
        std::swap(mc_, o.mc_);
        std::swap(pooled_, o.pooled_);
    }
    T* p_ = nullptr;
    size_t n_ = 0;
    MemCounter* mc_ = nullptr;
    bool pooled_ = false;
};

// distinct-column runs kept per streaming block (see DCsr::urun)
constexpr int kMaxRuns = 6;
constexpr int kRunWords = kMaxRuns + 2;

// CSR matrix resident on the device
struct DCsr {
    int n = 0, m = 0;
    int64_t nnz = 0;
    DBuf<int> rowptr, col;
    DBuf<double> val;
    DBuf<float> val32;
    // row blocks for the streaming SpMV: blk[b] .. blk[b+1] rows of block b;
    // `group` threads reduce each row (1 for short rows, 8 when rows are long)
    DBuf<int> blk;
    // blkk[b] = rowptr[blk[b]]: first stored entry of block b (nblk + 1
    // values), so a streaming block knows its entry range from its index
    DBuf<int> blkk;
    int nblk = 0;
    int group = 1;
    // packed columns for the streaming SpMV (when every row block's columns
    // span fewer than 2^16 values): col = cbase[b] + col16 within block b
    DBuf<uint16_t> col16;
    DBuf<int> cbase;
    int cap = 2048;  // most stored entries in one streaming block (kStreamCap or kStreamCapWide)
    // distinct columns of each packed streaming block, for staging the
    // gathered vector in LDS: block b's distinct packed columns, ascending,
    // are uoff[ustart[b] .. ustart[b+1]), and its entries' col16 then hold
    // indices into that list.  An empty list (more than unique_cap(cap)
    // distinct columns, or a block of one long row) leaves the block's col16
    // as column offsets, gathered from memory.
    DBuf<int> ustart;
    DBuf<uint16_t> uoff;
    int64_t nuniq = 0;  // total length of the lists
    // blocks whose distinct columns form at most kMaxRuns runs of consecutive
    // columns keep the runs instead of a list: urun[kRunWords b ..] = {runs,
    // distinct columns, then start | length << 16 per run}; runs = 0: none
    DBuf<uint32_t> urun;
    // the setup kernels' row blocks (at most kStreamCap entries) when the
    // streaming blocks above were widened; otherwise they share blk
    DBuf<int> sblk;
    int snblk = 0;
    const int* setup_blk() const { return sblk ? sblk.get() : blk.get(); }
    int setup_nblk() const { return sblk ? snblk : nblk; }
    // column bytes per stored entry the streaming kernels read
    double col_bytes() const { return col16 ? 2.0 : 4.0; }
    // bytes of the distinct-column lists and their block table
    double unique_bytes() const {
        return (ustart ? 2.0 * (double)nuniq + 4.0 * (nblk + 1) : 0.0) + (urun ? 4.0 * kRunWords * nblk : 0.0);
    }
};

constexpr int kBlock = 256;          // threads per block in streaming kernels
constexpr int kStreamCap = 2048;     // nnz staged in LDS per streaming block
// wider streaming blocks for large one-thread-per-row packed matrices: twice
// the bytes per workgroup (the setup kernels keep kStreamCap blocks)
constexpr int kStreamCapWide = 4096;
// most distinct columns of a streaming block of capacity `cap` staged in LDS
// (in the block's product array), and the reuse a block needs to be staged:
// at most kUniqueReusePct percent as many distinct columns as entries
constexpr int unique_cap(int cap) { return cap / 2; }
constexpr int kUniqueReusePct = 70;
// Widen a matrix's streaming blocks to kStreamCapWide when it has at least
// this many kStreamCap blocks.  A wide FP64 block's products take 32 KB of
// LDS, which halves the blocks a CU holds, and pays only on the largest
// operators; the finest operator (streamed by the FP64 outer CG in both
// forms) widens a little earlier.  A wide FP32 block takes the LDS of a
// narrow FP64 one, so the coarse operators of the FP32 form, streamed only
// in FP32, widen at half the size (measured on the 128^3 stack and the
// 96^3 cube: the fine FP32 smoother of the cube, 11.6k blocks, from 35.6 to
// 30.2 us; FP64 operators of 6.5k to 9.8k blocks 7 to 20% slower wide).
constexpr int kWideBlockMin = 12000;
constexpr int kWideBlockMinFine = 11000;
constexpr int kWideBlockMinFp32 = 6000;
constexpr int kMaxRowsPerBlock = kBlock;
constexpr int kLongRow = 96;         // setup kernels: longer single-row blocks take the whole-block path
constexpr int kWideRow = 32;         // streaming, one thread per row: wider rows are summed by 8 lanes of its wavefront
// rows longer than this are reduced by a whole block (a block of their own),
// for `group` threads per row
constexpr int long_row_limit(int group) { return group == 1 ? 256 : (32 * group < kStreamCap ? 32 * group : kStreamCap); }
// 8 threads per row instead of one (with 8-lane help for wide rows) on
// matrices that have rows longer than kLongRow and hold more than this share
// (in percent) of their entries in rows wider than kWideRow
constexpr int kGroup8WidePercent = 45;
constexpr int stream_group_rule(int max_len, int64_t wide_nnz, int64_t nnz) {
    return (max_len > kLongRow && wide_nnz * 100 > (int64_t)kGroup8WidePercent * nnz) ? 8 : 1;
}
// rows each group of `group` threads reduces in a block (one after the other)
constexpr int rows_per_group(int group) { return group == 1 ? 1 : 4; }
// most rows in one row block
constexpr int max_block_rows(int group) { return kBlock / group * rows_per_group(group); }

inline int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// pinned host memory of at least `bytes` (<= kReadbackBytes) owned by the
// calling thread, kept until the process ends: small read-backs through it
// take the direct DMA path instead of a staged copy into pageable memory
constexpr size_t kReadbackBytes = 64 << 10;
void* readback_buffer();

// synchronous device->host copy of a small array on a stream
template <typename T>
void d2h(T* host, const T* dev, size_t n, hipStream_t s) {
    if (n == 0) return;
    const size_t bytes = n * sizeof(T);
    if (bytes <= kReadbackBytes) {
        void* pin = readback_buffer();
        MATAMG_HIP(hipMemcpyAsync(pin, dev, bytes, hipMemcpyDeviceToHost, s));
        MATAMG_HIP(hipStreamSynchronize(s));
        std::memcpy(host, pin, bytes);
        return;
    }
    MATAMG_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s));
    MATAMG_HIP(hipStreamSynchronize(s));
}
template <typename T>
void h2d(T* dev, const T* host, size_t n, hipStream_t s) {
    if (n == 0) return;
    MATAMG_HIP(hipMemcpyAsync(dev, host, n * sizeof(T), hipMemcpyHostToDevice, s));
}

}  // namespace matamg
