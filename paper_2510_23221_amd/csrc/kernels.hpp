// Internal launchers shared by the C ABI translation units.
#pragma once

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

size_t cg_workspace_bytes(int64_t n, int m);

bko_status cg_solve(const Operator &op, int m, const double *B, int64_t ldb, double *X, int64_t ldx, double tol,
                    int max_iter, void *work, int *iters_host, bko_solve_info *info, hipStream_t stream);

}  // namespace bko
