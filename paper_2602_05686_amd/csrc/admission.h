// Host-only request bookkeeping of the solve server: the device-memory
// estimate that gates admission and the FIFO admission policy under a byte
// budget and a cap on concurrently admitted requests.  No HIP here, so the
// policy is testable on a host without a GPU.
#pragma once

#include <cstdint>
#include <deque>
#include <unordered_map>
#include <vector>

namespace matamg {

// Upper bound of the device bytes one request holds while its hierarchy is
// built (the setup peak), from the fine-level sizes.  Per stored entry of A:
// the matrix (12 B), strength values and drop mask (9 B), the strength
// numerators during the drop (8 B), the filtered matrix (12 B), the FP32
// copies (4 B), the SpGEMM products of the first level (bounded by 12 B) and
// the packed 16-bit columns of the operators and transfers (6 B);
// per node: coordinates, nodal and inverse tensors, aggregation state,
// tentative and smoothed prolongator rows, work and Krylov vectors; per
// element: the connectivity and tensors staged for the nodal averages; plus
// the dense coarsest inverse and its workspace for up to max_coarse unknowns.
inline int64_t estimate_setup_bytes(int64_t n, int64_t nnz, int64_t nelem, int npe, int dim, int max_coarse) {
    const int64_t ncomp = (int64_t)dim * (dim + 1) / 2;
    const int64_t per_nnz = 12 + 9 + 8 + 12 + 4 + 12 + 6;
    const int64_t per_node = 8 * dim + 16 * ncomp + 64 + 2 * 12 * 8 + 10 * 8 + 6 * 8 + 64;
    const int64_t per_elem = 4 * (int64_t)npe + 8 * (int64_t)dim * dim + 8 * (int64_t)npe;
    const int64_t nl = n < (int64_t)max_coarse ? n : (int64_t)max_coarse;
    const int64_t dense = 2 * 8 * nl * nl;
    const int64_t fixed = 16 << 20;
    return per_nnz * nnz + per_node * n + per_elem * nelem + dense + fixed;
}

// FIFO admission: the request at the head of the queue is admitted when
// its reservation fits in what the budget has left and a slot is free;
// later requests wait behind it (no overtaking, so no request starves).
class Admission {
  public:
    Admission(int64_t budget, int max_active) : budget_(budget), max_active_(max_active) {}

    int64_t budget() const { return budget_; }
    bool fits_ever(int64_t bytes) const { return bytes <= budget_; }
    int64_t used() const { return used_; }
    int64_t peak_used() const { return peak_used_; }
    int active() const { return (int)held_.size(); }
    size_t waiting() const { return queue_.size(); }

    void push(uint64_t id, int64_t bytes) { queue_.push_back({id, bytes}); }

    // admit from the head while it fits; returns the admitted ids in order
    std::vector<uint64_t> admit() {
        std::vector<uint64_t> out;
        while (!queue_.empty() && active() < max_active_ && used_ + queue_.front().bytes <= budget_) {
            const Entry e = queue_.front();
            queue_.pop_front();
            held_[e.id] = e.bytes;
            used_ += e.bytes;
            if (used_ > peak_used_) peak_used_ = used_;
            out.push_back(e.id);
        }
        return out;
    }

    // replace an admitted request's reservation (setup done: the estimate
    // becomes the bytes it keeps resident)
    void resize(uint64_t id, int64_t bytes) {
        auto it = held_.find(id);
        if (it == held_.end()) return;
        used_ += bytes - it->second;
        it->second = bytes;
        if (used_ > peak_used_) peak_used_ = used_;
    }

    void release(uint64_t id) {
        auto it = held_.find(id);
        if (it == held_.end()) return;
        used_ -= it->second;
        held_.erase(it);
    }

  private:
    struct Entry {
        uint64_t id;
        int64_t bytes;
    };
    int64_t budget_;
    int max_active_;
    int64_t used_ = 0, peak_used_ = 0;
    std::deque<Entry> queue_;
    std::unordered_map<uint64_t, int64_t> held_;
};

}  // namespace matamg
