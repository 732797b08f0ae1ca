// Multigrid hierarchy resident on one GPU, its setup driver, the V-cycle and
// the preconditioned CG driver.
#pragma once

#include <array>
#include <memory>

#include "common.h"
#include "kernels.h"

namespace matamg {

struct Level {
    DCsr A, P, R;  // operator; prolongator to / restriction from the next level
    DBuf<double> dinv;
    DBuf<float> dinv32;
    DBuf<double> x, sig;     // nodal coordinates [n][dim], tensors [n][ncomp]
    DBuf<uint8_t> dir, mask;
    DBuf<double> S;
    DBuf<int> agg;
    int nc = 0, mis_rounds = 0;
    double lam_pf = 0.0, omega = 0.0, lam_cheb = 0.0;
    std::vector<double> c1, c2;  // smoother step coefficients
    // V-cycle work vectors (b: right-hand side, x/x2: iterate double buffer,
    // d: smoother direction, r: residual)
    DBuf<double> b, xa, xb, d, r;
    DBuf<float> fb, fxa, fxb, fd, fr;
};

struct Hierarchy {
    amg_options opt{};
    int nlev = 0;
    std::array<Level, 16> lev;
    int nL = 0;
    DBuf<double> Ainv;  // dense inverse of the coarsest operator
    MemCounter mem;
    DBuf<double> scal;       // device scalars (see Scalar)
    DBuf<double> partial;    // reduction partials
    DBuf<unsigned> counter;  // reduction counters
    DBuf<double> cr, cz, cp, cq, cx, cb;  // CG vectors (x, b used for host inputs)
    double* hscal = nullptr; // pinned host mirror of scal
    hipStream_t ws = nullptr;        // the solve's own stream (graphs cannot capture the null stream)
    hipEvent_t ev_in = nullptr;      // orders the solve after the caller's stream
    hipGraphExec_t graph[2] = {nullptr, nullptr};  // captured CG steps, by parity
    bool use_graphs = true;
    double t_setup = 0.0;
    double t_update = 0.0;   // duration of the last update_values
    bool fp32 = false;

    ~Hierarchy();
    DotTarget dt(int slot) const;
    void vcycle(const double* r, double* z, DotTarget rz, hipStream_t s);
    template <typename T>
    void vcycle_t(const double* r, double* z, DotTarget rz, hipStream_t s);
    double vcycle_alg_bytes() const;
    double time_smoother(int level, int reps, hipStream_t s, double* bytes_per_launch);
    hipGraphExec_t step_graph(int cur);
    void ensure_solve_resources();
    void release_setup_data();
};

// device scalar slots
enum Scalar { S_RZ0 = 0, S_RZ1 = 1, S_PQ = 2, S_RR = 3, S_BB = 4, S_TMP = 5, S_NSCAL = 8 };

// wide_blocks: give large finest-level operators the wider streaming blocks
// (the batched launches of the server take only kStreamCap blocks)
std::unique_ptr<Hierarchy> build_hierarchy(int64_t n, const int* rowptr, const int* col, const double* val,
                                           int64_t nelem, int npe, const int* elem_nodes,
                                           const double* elem_sigma, const double* coords,
                                           const amg_options& opt, bool host_ptrs, hipStream_t s,
                                           bool wide_blocks = true);

// new values of A on the setup's pattern; masks, aggregates, coordinates and
// tensors are kept, every value-dependent quantity is recomputed
void update_values(Hierarchy& h, const double* val, bool host_ptrs, hipStream_t s);

amg_status pcg_solve(Hierarchy& h, const double* b, double* x, double tol, int max_iter, bool host_ptrs,
                     hipStream_t s, amg_solve_info* info);

// Workspace of one PCG solve: the iterate x (in/out) and r, z, p, q
// (device vectors of the finest size), the device scalars (S_NSCAL), the
// reduction partials and counter, a host mirror of the scalars, the stream,
// and whether the captured step graphs may run (only with the hierarchy's
// own buffers, which they hold).
struct PcgWork {
    double *x, *r, *z, *p, *q;
    double* scal;
    double* partial;
    unsigned* counter;
    double* hscal;
    hipStream_t stream;
    bool graphs;
};
// the PCG iteration of pcg_solve on a given workspace; allocates nothing
amg_status pcg_run(Hierarchy& h, const PcgWork& w, const double* b, double tol, int max_iter, int* iters,
                   double* rel_true);
// doubles of reduction partials a solve on h needs
size_t pcg_partials(const Hierarchy& h);

// PCG with its workspace in the library's fixed device array (noalloc.hip):
// device b and x (x iterated in place), the caller's stream, no allocation
amg_status pcg_solve_noalloc(Hierarchy& h, const double* b, double* x, double tol, int max_iter, hipStream_t s,
                             amg_solve_info* info);
size_t noalloc_need_bytes(const Hierarchy& h);
size_t noalloc_scratch_bytes();

}  // namespace matamg
