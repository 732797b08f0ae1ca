// Solve server: continuous batching of many AMG-preconditioned CG solves on
// one GPU.  Requests are admitted in arrival order under a device-memory
// budget, their hierarchies are built by setup workers (one stream each)
// while admitted solves keep iterating, and every CG step of all solving
// requests runs as one sequence of batched launches on the engine stream.
#pragma once

#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "admission.h"
#include "hierarchy.h"

namespace matamg {

struct Request {
    uint64_t id = 0;
    int64_t n = 0, nnz = 0, nelem = 0;
    int npe = 0;
    std::vector<int> rowptr, col, elem_nodes;
    std::vector<double> val, elem_sigma, coords, b, x0;
    double tol = 1e-8;
    int max_iter = 1000;
    int64_t est = 0, setup_peak = 0, resident = 0;
    double t_arrival = 0, t_admit = 0, t_setup_done = 0, t_done = 0;
    amg_status status = AMG_OK;
    std::string error;
    bool done = false;
    std::unique_ptr<Hierarchy> h;
    // CG state (mirrors the one-hierarchy solver)
    int slot = -1;
    int cur = S_RZ0;
    bool first = true;
    int iters = 0;
    double bn = 0.0, rel_true = 0.0;
    int max_batch = 0;
    int levels = 0;
    std::vector<double> x;
};

struct ServerStats {
    int64_t submitted = 0, completed = 0, failed = 0, rejected = 0;
    int64_t steps = 0, launches = 0, batch_sum = 0, max_batch = 0;
    int64_t estimate_exceeded = 0;
};

class Server {
  public:
    Server(const amg_options& opt, int64_t budget, int max_active, int setup_workers);
    ~Server();
    // copies the inputs; returns AMG_ERR_BUDGET if the request can never fit
    amg_status submit(int64_t n, const int* rowptr, const int* col, const double* val, int64_t nelem, int npe,
                      const int* elem_nodes, const double* elem_sigma, const double* coords, const double* b,
                      const double* x0, double tol, int max_iter, uint64_t* id);
    // ids of finished requests (waits up to timeout_s for the first one)
    int poll(uint64_t* ids, int cap, double timeout_s);
    // hands over a finished request (once) and forgets it
    std::unique_ptr<Request> take(uint64_t id);
    void stats(ServerStats* st, int64_t* budget, int64_t* used, int64_t* peak_used, int* active, int64_t* waiting);
    double now() const;
    // an idle engine waits up to this long for requests still in setup
    // before it starts solving the ready ones (0: start at once)
    void set_batch_wait(double seconds);

  private:
    void worker_main();
    void engine_main();
    void admit_locked();
    void finish_locked(Request* r);
    template <typename T>
    void run_step(std::vector<Request*>& batch);

    amg_options opt_;
    int device_ = 0;
    int max_active_;
    double t0_;
    std::mutex mu_;
    std::condition_variable cv_setup_, cv_engine_, cv_done_;
    Admission adm_;
    std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs_;
    std::deque<Request*> setup_q_;
    std::vector<Request*> ready_;
    std::deque<uint64_t> done_q_;
    uint64_t next_id_ = 1;
    bool stop_ = false;
    int in_setup_ = 0;         // admitted requests whose setup has not finished
    double batch_wait_ = 0.0;
    ServerStats st_;
    std::vector<std::thread> workers_;
    std::thread engine_;
    // engine-owned device state
    hipStream_t es_ = nullptr;
    DBuf<double> sscal_;     // [max_active][S_NSCAL] CG scalars per slot
    double* hsc_ = nullptr;  // pinned mirror
    std::vector<int> free_slots_;
    DBuf<unsigned char> dtab_;        // descriptor tables of one step
    unsigned char* htab_ = nullptr;   // pinned staging
    size_t htab_cap_ = 0;
};

}  // namespace matamg
