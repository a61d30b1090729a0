// Internal launchers shared by the C ABI translation units.
#pragma once

#include <map>
#include <utility>
#include <vector>

#include "common.hpp"

namespace bko {

// y = A x (or y = b - A x) over m columns, matrix-free variable-coefficient
// 5/7-point stencil.  t_in / t_out / compute are bko_dtype values.
bko_status launch_stencil(const Operator &op, int m, const void *X, int64_t ldx, bko_dtype t_in,
                          void *Y, int64_t ldy, bko_dtype t_out, bko_dtype compute,
                          const double *Bres, int64_t ldb, hipStream_t stream, const int *skip = nullptr,
                          int *stop = nullptr);

bko_status launch_combine(int64_t n, int s, int64_t m, const void *X, int64_t ldx, bko_dtype x_t,
                          const void *C, int64_t ldc, bko_dtype c_t, void *T, int64_t ldt,
                          bko_dtype t_t, bko_dtype compute, hipStream_t stream);

// zero-fill bytes (a kernel, never a memset node, so it is safe in graphs)
bko_status launch_zero(void *p, size_t bytes, hipStream_t stream);

size_t solve_workspace_bytes(int64_t n, int s, bko_dtype compute);

bko_status block_solve(const Operator &op, int s, const double *B, int64_t ldb, double *X,
                       int64_t ldx, const double *X0, int64_t ldx0, bko_dtype compute, double tol,
                       int max_iter, void *work, size_t work_bytes, bko_solve_info *info,
                       hipStream_t stream);

// Captured iteration chunks of a batch plan (keyed by chunk length), valid
// for one workspace address.
struct GraphCache {
    void *work = nullptr;
    std::map<int, hipGraphExec_t> execs;
    void clear()
    {
        for (auto &kv : execs) (void)hipGraphExecDestroy(kv.second);
        execs.clear();
        work = nullptr;
    }
    ~GraphCache() { clear(); }
};

// A batch of chips solved together (one s and compute dtype for all).
struct BatchPlan {
    std::vector<const Operator *> ops;
    int s = 0;
    bko_dtype compute = BKO_F64;
    int wg_cap = 512;   // per-chip workgroups of the row kernels (autotuned)
    bool tuned = false;
    std::vector<std::pair<int, float>> tune_ms;  // (cap, ms per timed pass)
    GraphCache graphs;
};

size_t batch_workspace_bytes(const BatchPlan &p);
bko_status batch_tune(BatchPlan &p, void *work, hipStream_t stream);
bko_status batch_solve(BatchPlan &p, const double *const *B, const int64_t *ldb, double *const *X,
                       const int64_t *ldx, const double *const *X0, const int64_t *ldx0, double tol,
                       int max_iter, void *work, bko_solve_info *infos, hipStream_t stream);

size_t cg_workspace_bytes(int64_t n, int m);

bko_status cg_solve(const Operator &op, int m, const double *B, int64_t ldb, double *X, int64_t ldx, double tol,
                    int max_iter, void *work, int *iters_host, bko_solve_info *info, hipStream_t stream);

}  // namespace bko
