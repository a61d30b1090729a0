// Matrix-free variable-coefficient 5/7-point stencil over blocks of fields:
// Y[:, c] = A X[:, c]  (operator action, Sec. III-C, Eq. (6), and the block
// product inside the block solve, Sec. III-A), or Y = B - A X (residual).
//
// A is stored as its diagonal and the three forward-face couplings of every
// cell (wx[a] couples a with a+1, wy[a] with a+nx, wz[a] with a+nx*ny; zero
// where the neighbour is outside the grid), so
//   (A x)_a = diag_a x_a - wx_a x_{a+1} - wx_{a-1} x_{a-1}
//                        - wy_a x_{a+nx} - wy_{a-nx} x_{a-nx}
//                        - wz_a x_{a+p} - wz_{a-p} x_{a-p},     p = nx*ny.
//
// Work decomposition: a workgroup owns kTile consecutive cells and a group of
// columns; each thread loads its cell's seven coefficients once and reuses
// them for every column of the group.  The workgroup order is remapped so
// that each XCD walks a contiguous range of (column group, cell tile) pairs,
// keeping the neighbouring tiles that supply the y / z halo in one L2.
#include "kernels.hpp"

namespace bko {

namespace {

constexpr int kThreads = 256;

template <class Tin, class Tout, class Tc, class Acc, bool kResidual>
__global__ __launch_bounds__(kThreads) void stencil_kernel(
    const Tc *__restrict__ diag, const Tc *__restrict__ wx, const Tc *__restrict__ wy,
    const Tc *__restrict__ wz, int nx, int ny, int nz, const Tin *__restrict__ X, int64_t ldx,
    Tout *__restrict__ Y, int64_t ldy, const double *__restrict__ Bres, int64_t ldb, int m,
    int cols_per_group, uint32_t ntiles, uint32_t nblocks, const int *__restrict__ skip, int *stop)
{
    if (skip && *skip) {
        // the iteration before this one converged: tell the later kernels
        if (stop && blockIdx.x == 0 && threadIdx.x == 0) *stop = 1;
        return;
    }
    const uint32_t lb = remap_block(blockIdx.x, nblocks);
    const uint32_t tile = lb % ntiles;
    const uint32_t group = lb / ntiles;
    const int64_t plane = static_cast<int64_t>(nx) * ny;
    const int64_t n = plane * nz;
    const int64_t a = static_cast<int64_t>(tile) * kThreads + threadIdx.x;
    if (a >= n) return;
    const int i = static_cast<int>(a % nx);
    const int64_t q = a / nx;
    const int j = static_cast<int>(q % ny);
    const int l = static_cast<int>(q / ny);

    // neighbour offsets; a missing neighbour reads the cell itself with a
    // zero coupling so every load stays inside the column
    const int64_t oxm = i > 0 ? -1 : 0, oxp = i < nx - 1 ? 1 : 0;
    const int64_t oym = j > 0 ? -static_cast<int64_t>(nx) : 0, oyp = j < ny - 1 ? nx : 0;
    const int64_t ozm = l > 0 ? -plane : 0, ozp = l < nz - 1 ? plane : 0;
    const Acc d = static_cast<Acc>(diag[a]);
    const Acc cxp = static_cast<Acc>(wx[a]);
    const Acc cxm = i > 0 ? static_cast<Acc>(wx[a - 1]) : Acc(0);
    const Acc cyp = static_cast<Acc>(wy[a]);
    const Acc cym = j > 0 ? static_cast<Acc>(wy[a - nx]) : Acc(0);
    const Acc czp = static_cast<Acc>(wz[a]);
    const Acc czm = l > 0 ? static_cast<Acc>(wz[a - plane]) : Acc(0);

    const int c0 = static_cast<int>(group) * cols_per_group;
    const int c1 = min(m, c0 + cols_per_group);
    for (int c = c0; c < c1; ++c) {
        const Tin *x = X + static_cast<int64_t>(c) * ldx + a;
        const Acc xc = load_as<Acc>(x);
        const Acc nb = cxm * load_as<Acc>(x + oxm) + cxp * load_as<Acc>(x + oxp) +
                       cym * load_as<Acc>(x + oym) + cyp * load_as<Acc>(x + oyp) +
                       czm * load_as<Acc>(x + ozm) + czp * load_as<Acc>(x + ozp);
        Acc y = d * xc - nb;
        if constexpr (kResidual) y = static_cast<Acc>(Bres[static_cast<int64_t>(c) * ldb + a]) - y;
        Y[static_cast<int64_t>(c) * ldy + a] = store_from<Tout, Acc>(y);
    }
}

template <class Tin, class Tout, class Tc, class Acc, bool kResidual>
bko_status run(const Operator &op, const Tc *diag, const Tc *wx, const Tc *wy, const Tc *wz, int m,
               const void *X, int64_t ldx, void *Y, int64_t ldy, const double *Bres, int64_t ldb,
               hipStream_t stream, const int *skip, int *stop)
{
    const uint32_t ntiles = static_cast<uint32_t>((op.n + kThreads - 1) / kThreads);
    // enough column groups to fill the chip, few enough that each thread
    // reuses its coefficients over several columns
    int cols = 8;
    if (static_cast<int64_t>(ntiles) * ((m + cols - 1) / cols) < 4096) cols = 1;
    const uint32_t ngroups = static_cast<uint32_t>((m + cols - 1) / cols);
    const uint64_t nb = static_cast<uint64_t>(ntiles) * ngroups;
    if (nb > 0x7fffffffu) {
        set_error("stencil grid of %llu workgroups too large", (unsigned long long)nb);
        return BKO_EINVAL;
    }
    hipLaunchKernelGGL((stencil_kernel<Tin, Tout, Tc, Acc, kResidual>), dim3(static_cast<uint32_t>(nb)),
                       dim3(kThreads), 0, stream, diag, wx, wy, wz, op.nx, op.ny, op.nz,
                       static_cast<const Tin *>(X), ldx, static_cast<Tout *>(Y), ldy, Bres, ldb, m, cols,
                       ntiles, static_cast<uint32_t>(nb), skip, stop);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

template <class Tin, class Tout>
bko_status dispatch_compute(const Operator &op, int m, const void *X, int64_t ldx, void *Y, int64_t ldy,
                            bko_dtype compute, hipStream_t stream, const int *skip, int *stop)
{
    if (compute == BKO_F64)
        return run<Tin, Tout, double, double, false>(op, op.diag64, op.wx64, op.wy64, op.wz64, m, X, ldx, Y,
                                                     ldy, nullptr, 0, stream, skip, stop);
    return run<Tin, Tout, float, float, false>(op, op.diag32, op.wx32, op.wy32, op.wz32, m, X, ldx, Y, ldy,
                                               nullptr, 0, stream, skip, stop);
}

template <class Tin>
bko_status dispatch_out(const Operator &op, int m, const void *X, int64_t ldx, void *Y, int64_t ldy,
                        bko_dtype t_out, bko_dtype compute, hipStream_t stream, const int *skip, int *stop)
{
    switch (t_out) {
    case BKO_F64: return dispatch_compute<Tin, double>(op, m, X, ldx, Y, ldy, compute, stream, skip, stop);
    case BKO_F32: return dispatch_compute<Tin, float>(op, m, X, ldx, Y, ldy, compute, stream, skip, stop);
    default: return dispatch_compute<Tin, bf16>(op, m, X, ldx, Y, ldy, compute, stream, skip, stop);
    }
}

}  // namespace

bko_status launch_stencil(const Operator &op, int m, const void *X, int64_t ldx, bko_dtype t_in, void *Y,
                          int64_t ldy, bko_dtype t_out, bko_dtype compute, const double *Bres, int64_t ldb,
                          hipStream_t stream, const int *skip, int *stop)
{
    if (m <= 0) return BKO_OK;
    if (Bres != nullptr) {
        // residual form is FP64 only
        return run<double, double, double, double, true>(op, op.diag64, op.wx64, op.wy64, op.wz64, m, X, ldx, Y,
                                                         ldy, Bres, ldb, stream, skip, stop);
    }
    switch (t_in) {
    case BKO_F64: return dispatch_out<double>(op, m, X, ldx, Y, ldy, t_out, compute, stream, skip, stop);
    case BKO_F32: return dispatch_out<float>(op, m, X, ldx, Y, ldy, t_out, compute, stream, skip, stop);
    default: return dispatch_out<bf16>(op, m, X, ldx, Y, ldy, t_out, compute, stream, skip, stop);
    }
}

}  // namespace bko
