// Internal launchers shared by the C ABI translation units.
#pragma once

#include <map>
#include <string>
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
// The operator action of several chips in one grouped launch (chips whose
// rows or views do not suit the tiled kernel get a launch of their own).
// m[c] fields of chip c; jobs_dev: stencil_group_job_bytes(nchips) bytes of
// device memory for the job table, copied from host_jobs (which must live
// until the stream has passed the launch).  ty_cap > 0 caps the tile height.
size_t stencil_group_job_bytes(int nchips);
bko_status launch_stencil_group(const Operator *const *ops, int nchips, const int *m, const void *const *X,
                                const int64_t *ldx, bko_dtype t_in, void *const *Y, const int64_t *ldy,
                                bko_dtype t_out, bko_dtype compute, int ty_cap, void *jobs_dev,
                                std::vector<unsigned char> &host_jobs, hipStream_t stream);
// Rows per tile the operator action takes for these fields (0: per-cell kernel).
int stencil_tile_rows(const Operator &op, int m, const void *X, int64_t ldx, bko_dtype t_in, const void *Y,
                      int64_t ldy, bko_dtype t_out, bko_dtype compute);

// `sweeps` damped Jacobi sweeps X <- X + omega (B - A X) / diag(A) in FP64
// over m columns; work is an n x m FP64 block (ldw >= n).
bko_status launch_jacobi(const Operator &op, int m, const double *B, int64_t ldb, double *X, int64_t ldx,
                         double *work, int64_t ldw, int sweeps, double omega, hipStream_t stream);

bko_status launch_combine(int64_t n, int s, int64_t m, const void *X, int64_t ldx, bko_dtype x_t,
                          const void *C, int64_t ldc, bko_dtype c_t, void *T, int64_t ldt,
                          bko_dtype t_t, bko_dtype compute, hipStream_t stream);
// T = X C + E in FP64, E the counter-based noise of (seed, field_offset + f, cell).
bko_status launch_combine_noisy(int64_t n, int s, int64_t m, const double *X, int64_t ldx, const double *C, int64_t ldc,
                                double *T, int64_t ldt, int kind, double amp, uint64_t seed, uint64_t field_offset,
                                hipStream_t stream);
bko_status launch_noise_fill(int64_t n, int64_t m, double *E, int64_t lde, int kind, double amp, uint64_t seed,
                             uint64_t field_offset, hipStream_t stream);
// alpha = mu / sum(mu) per field in place; fields with |sum| < min_abs are
// left as they are, flags[j] = 1 for them and 0 for the others (device).
bko_status launch_normalize_weights(int s, int64_t m, double *C, int64_t ldc, double min_abs, int *flags,
                                    hipStream_t stream);
// T = X C and F = Y C in FP64 with one pass over the fields (Y = A X).
bko_status launch_combine_dual(int64_t n, int s, int64_t m, const double *X, int64_t ldx, const double *Y, int64_t ldy,
                               const double *C, int64_t ldc, double *T, int64_t ldt, double *F, int64_t ldf,
                               hipStream_t stream);

// T = X C for several chips in one grouped launch (X, C FP64; T of t_t),
// m[c] fields of chip c; fields_per_wg > 0 fixes the fields per workgroup.
// jobs_dev: combine_group_job_bytes(nchips) bytes of device memory, copied
// from host_jobs (which must live until the stream has passed the launch).
size_t combine_group_job_bytes(int nchips);
bko_status launch_combine_group(int nchips, const int64_t *n, int s, const int *m, const double *const *X,
                                const int64_t *ldx, const double *const *C, const int64_t *ldc, void *const *T,
                                const int64_t *ldt, bko_dtype t_t, bko_dtype compute, int64_t fields_per_wg,
                                void *jobs_dev, std::vector<unsigned char> &host_jobs, hipStream_t stream);

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
    int tiles_per_wg = 1;  // row tiles per workgroup of the row kernels (autotuned)
    bool tuned = false;
    std::vector<std::pair<int, float>> tune_ms;  // (tiles per workgroup, ms of the timed passes)
    GraphCache graphs;
    // outputs (bko_batch_run): fields per chip (empty: the plan only solves),
    // combination arithmetic, T and F storage types, the operator action's
    // arithmetic, and the two output knobs (0 = the launcher's default),
    // chosen by timing on the first run
    std::vector<int> m;
    bko_dtype comb_compute = BKO_F64, t_dtype = BKO_F64, f_dtype = BKO_F64, apply_compute = BKO_F64;
    int out_ty_cap = 0;
    int64_t out_fields_per_wg = 0;
    bool out_tuned = false;
    std::vector<std::pair<std::string, float>> out_tune_ms;  // (candidate, ms)
};

// Bytes of the solve's part of a batch workspace, and of the whole
// workspace (the solve's part, then the output job tables).
size_t batch_solve_bytes(const BatchPlan &p);
size_t batch_workspace_bytes(const BatchPlan &p);
bko_status batch_tune(BatchPlan &p, void *work, hipStream_t stream);
bko_status batch_solve(BatchPlan &p, const double *const *B, const int64_t *ldb, double *const *X,
                       const int64_t *ldx, const double *const *X0, const int64_t *ldx0, double tol,
                       int max_iter, void *work, bko_solve_info *infos, hipStream_t stream);

// ---- learned start (convolutional encoder-decoder)
bko_status nn_conv(const float *A, int Ca, const float *B, int Cb, int mode, int N, int H, int W, int Co, int K,
                   const uint16_t *wgt, int transposed, const float *bias, float *out, int relu, hipStream_t st);
// the forward convolution on the BF16 matrix cores (BF16 inputs, FP32 accumulation)
bko_status nn_conv_mfma(const float *A, int Ca, const float *B, int Cb, int mode, int N, int H, int W, int Co, int K,
                        const uint16_t *wgt, const float *bias, float *out, int relu, hipStream_t st);
size_t nn_wgrad_part_floats(int N, int H, int W, int Ci, int Co, int K);
bko_status nn_wgrad(const float *A, int Ca, const float *B, int Cb, int mode, const float *g, int N, int H, int W,
                    int Co, int K, float *part, float *gw, float *gb, hipStream_t st);
bko_status nn_relu_bwd(float *g, const float *y, int64_t n, hipStream_t st);
bko_status nn_pool_bwd(const float *g, int NC, int H, int W, const float *add, float *gA, hipStream_t st);
bko_status nn_upcat_bwd(const float *g, int N, int Ca, int Cb, int H, int W, float *gA, float *gB, hipStream_t st);
int nn_mse_blocks(int64_t n);
bko_status nn_mse(const float *pred, const float *target, int64_t n, float *grad, float *lpart, hipStream_t st);
bko_status nn_adam(float *p, const float *g, float *m, float *v, uint16_t *pb, int64_t n, float lr, int t,
                   hipStream_t st);
bko_status nn_to_bf16(const float *p, uint16_t *pb, int64_t n, hipStream_t st);
bko_status lstart_pack(int nx, int ny, int nz, const double *F, int64_t ldf, int m, const double *kc, float kmu,
                       float ksig, float hval, double *scale, float *x, hipStream_t st);
bko_status lstart_pack_target(int64_t n, const double *T, int64_t ldt, int m, const double *scale, double gain,
                              float *t, hipStream_t st);
bko_status lstart_unpack(int64_t n, const float *y, int m, const double *scale, double gain, double *X0, int64_t ldx,
                         hipStream_t st);

// The 4-level encoder-decoder (layer table in nn.hip).  Host metadata; the
// caller owns the state buffer (parameters, gradients, Adam moments, BF16
// copy) and the activation workspace.
struct UNet {
    struct Layer {
        int ci, co, k, relu, h, w;
        int64_t woff, boff;
        size_t act, grad;  // workspace offsets (floats)
    };
    struct State {
        float *params, *grads, *m, *v;
        uint16_t *pb;
    };
    int cin, cout, base, H, W, batch;
    Layer L[15];
    int64_t nparams = 0;
    size_t scratch_off = 0, skip_off[3] = {0, 0, 0}, part_off = 0, lpart_off = 0, work_floats = 0;
    int step = 0;

    UNet(int cin, int cout, int base, int H, int W, int batch);
    size_t state_bytes() const;
    State state(void *p) const;
    bko_status set_params(void *state, const float *params, hipStream_t st);
    // mfma: the convolutions on the BF16 matrix cores (inference)
    bko_status forward(void *state, void *work, const float *x, int n, float *y, hipStream_t st,
                       bool mfma = false) const;
    bko_status gradient(void *state, void *work, const float *x, const float *target, int n, float *loss,
                        hipStream_t st) const;
    bko_status adam(void *state, float lr, hipStream_t st);
};

size_t cg_workspace_bytes(int64_t n, int m);

bko_status cg_solve(const Operator &op, int m, const double *B, int64_t ldb, double *X, int64_t ldx, double tol,
                    int max_iter, void *work, int *iters_host, bko_solve_info *info, hipStream_t stream);

}  // namespace bko
