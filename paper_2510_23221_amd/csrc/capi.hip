// C ABI entry points: argument validation, operator handles, assembly of the
// cell-centred heat operator, timing hooks.  Every entry point catches
// everything so no C++ exception crosses the ABI.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "kernels.hpp"

namespace bko {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

bko_status hip_fail(hipError_t e, const char *what)
{
    set_error("HIP error %d (%s) in %s", static_cast<int>(e), hipGetErrorString(e), what);
    return BKO_EHIP;
}

size_t device_max_lds()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) return 65536;
    return static_cast<size_t>(v);
}

int device_cu_count()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) return 256;
    return v;
}

CoeffLayout coeff_layout(int64_t n)
{
    CoeffLayout L{};
    size_t off = 0;
    for (int a = 0; a < 4; ++a) {
        L.off[a] = off;
        off = align_up(off + sizeof(double) * static_cast<size_t>(n), 256);
    }
    for (int a = 4; a < 8; ++a) {
        L.off[a] = off;
        off = align_up(off + sizeof(float) * static_cast<size_t>(n), 256);
    }
    for (int a = 8; a < 12; ++a) {
        L.off[a] = off;
        off = align_up(off + sizeof(double) * static_cast<size_t>(n), 256);
    }
    for (int a = 12; a < 16; ++a) {
        L.off[a] = off;
        off = align_up(off + sizeof(float) * static_cast<size_t>(n), 256);
    }
    L.off[16] = off;
    off = align_up(off + sizeof(double) * static_cast<size_t>(n), 256);
    L.status_off = off;
    L.bytes = off + 256;
    return L;
}

// ------------------------------------------------------------ timing hooks

namespace {
struct TimingState {
    std::mutex mu;
    unsigned mask = 0;  // timed families, bit f = family f
    std::vector<hipEvent_t> pool;
    struct Pair { int family; hipEvent_t a, b; };
    std::vector<Pair> pending;
    int launches[kNumFamilies] = {};
    double total_ms[kNumFamilies] = {};
    unsigned stride = 1;                  // time one launch in every `stride` of a family
    unsigned counter[kNumFamilies] = {};  // launches seen per family
};
TimingState &timing()
{
    static TimingState *t = new TimingState();  // never destroyed: events may outlive statics
    return *t;
}
hipEvent_t take_event(TimingState &t)
{
    if (!t.pool.empty()) {
        hipEvent_t e = t.pool.back();
        t.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
bko_status drain(TimingState &t)
{
    for (auto &p : t.pending) {
        float ms = 0.f;
        BKO_HIP(hipEventSynchronize(p.b));
        BKO_HIP(hipEventElapsedTime(&ms, p.a, p.b));
        t.launches[p.family] += 1;
        t.total_ms[p.family] += ms;
        t.pool.push_back(p.a);
        t.pool.push_back(p.b);
    }
    t.pending.clear();
    return BKO_OK;
}
}  // namespace

bool timing_active() { return timing().mask != 0; }

TimedLaunch::TimedLaunch(int fam, hipStream_t s) : family(fam), stream(s), ev0(nullptr), ev1(nullptr), in_dispatch(false)
{
    TimingState &t = timing();
    if (!(t.mask & (1u << fam))) return;
    std::lock_guard<std::mutex> g(t.mu);
    if (t.counter[fam]++ % t.stride != 0) return;
    hipEvent_t a = take_event(t), b = take_event(t);
    if (!a || !b) {
        if (a) t.pool.push_back(a);
        if (b) t.pool.push_back(b);
        return;
    }
    // the start marker; launch() re-records it inside the kernel's dispatch
    if (hipEventRecord(a, s) == hipSuccess) {
        ev0 = a;
        ev1 = b;
    } else {
        t.pool.push_back(a);
        t.pool.push_back(b);
    }
}

TimedLaunch::~TimedLaunch()
{
    if (!ev0) return;
    TimingState &t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    hipEvent_t b = static_cast<hipEvent_t>(ev1);
    if (in_dispatch || hipEventRecord(b, stream) == hipSuccess) {
        t.pending.push_back({family, static_cast<hipEvent_t>(ev0), b});
        if (t.pending.size() > 4096) drain(t);
    } else {
        t.pool.push_back(static_cast<hipEvent_t>(ev0));
        t.pool.push_back(b);
    }
}

// ------------------------------------------------------------ assembly

__device__ inline double face_interior(double ka, double kb, double d2)
{
    // symmetric in (ka, kb) bit for bit: order the operands
    const double lo = fmin(ka, kb), hi = fmax(ka, kb);
    return 2.0 * lo * hi / ((lo + hi) * d2);
}

__device__ inline double face_boundary(int kind, double ka, double d, double h)
{
    if (kind == BKO_BC_DIRICHLET0) return 2.0 * ka / (d * d);
    if (kind == BKO_BC_ROBIN) return 1.0 / (d * (d / (2.0 * ka) + 1.0 / h));
    return 0.0;
}

struct FaceSpec {
    int bc[6];
    double h[6];
    double d[3];
};

__global__ __launch_bounds__(256) void assemble_kernel(int nx, int ny, int nz, FaceSpec fs,
                                                       const double *__restrict__ k, double *diag64,
                                                       double *wx64, double *wy64, double *wz64,
                                                       float *diag32, float *wx32, float *wy32,
                                                       float *wz32, int *bad)
{
    const int64_t n = static_cast<int64_t>(nx) * ny * nz;
    const int64_t a = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const int64_t plane = static_cast<int64_t>(nx) * ny;
    const int i = static_cast<int>(a % nx);
    const int j = static_cast<int>((a / nx) % ny);
    const int l = static_cast<int>(a / plane);
    const double ka = k[a];
    if (!(ka > 0.0) || !isfinite(ka)) atomicAdd(bad, 1);
    const int idx[3] = {i, j, l};
    const int dims[3] = {nx, ny, nz};
    const int64_t stride[3] = {1, nx, plane};
    double plus[3];
    double diag = 0.0;
    for (int ax = 0; ax < 3; ++ax) {
        const double d = fs.d[ax];
        const double d2 = d * d;
        if (idx[ax] > 0) diag += face_interior(ka, k[a - stride[ax]], d2);
        else diag += face_boundary(fs.bc[2 * ax], ka, d, fs.h[2 * ax]);
        if (idx[ax] < dims[ax] - 1) {
            plus[ax] = face_interior(ka, k[a + stride[ax]], d2);
            diag += plus[ax];
        } else {
            plus[ax] = 0.0;
            diag += face_boundary(fs.bc[2 * ax + 1], ka, d, fs.h[2 * ax + 1]);
        }
    }
    diag64[a] = diag;
    wx64[a] = plus[0];
    wy64[a] = plus[1];
    wz64[a] = plus[2];
    diag32[a] = static_cast<float>(diag);
    wx32[a] = static_cast<float>(plus[0]);
    wy32[a] = static_cast<float>(plus[1]);
    wz32[a] = static_cast<float>(plus[2]);
}

// The symmetrically scaled operator S A S with S = diag(A)^(-1/2) (the
// Jacobi preconditioner applied on both sides, which keeps the operator
// symmetric): diagonal d s^2, forward coupling w_ab s_a s_b.
__global__ void scale_coeff_kernel(int nx, int ny, int nz, const double *__restrict__ diag,
                                   const double *__restrict__ wx, const double *__restrict__ wy,
                                   const double *__restrict__ wz, double *__restrict__ sdiag64,
                                   double *__restrict__ swx64, double *__restrict__ swy64,
                                   double *__restrict__ swz64, float *__restrict__ sdiag32, float *__restrict__ swx32,
                                   float *__restrict__ swy32, float *__restrict__ swz32, double *__restrict__ scale)
{
    const int64_t plane = static_cast<int64_t>(nx) * ny;
    const int64_t n = plane * nz;
    const int64_t a = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const int i = static_cast<int>(a % nx);
    const int j = static_cast<int>((a / nx) % ny);
    const int l = static_cast<int>(a / plane);
    const double sa = 1.0 / sqrt(diag[a]);
    // a coupling to a missing neighbour is zero; its partner's scale is unused
    const double sx = i < nx - 1 ? 1.0 / sqrt(diag[a + 1]) : 0.0;
    const double sy = j < ny - 1 ? 1.0 / sqrt(diag[a + nx]) : 0.0;
    const double sz = l < nz - 1 ? 1.0 / sqrt(diag[a + plane]) : 0.0;
    const double d = diag[a] * sa * sa;
    const double cx = wx[a] * sa * sx, cy = wy[a] * sa * sy, cz = wz[a] * sa * sz;
    scale[a] = sa;
    sdiag64[a] = d;
    swx64[a] = cx;
    swy64[a] = cy;
    swz64[a] = cz;
    sdiag32[a] = static_cast<float>(d);
    swx32[a] = static_cast<float>(cx);
    swy32[a] = static_cast<float>(cy);
    swz32[a] = static_cast<float>(cz);
}

// g_a = sum over the boundary faces of cell a of w_face u_face (Sec. II-A's
// nonhomogeneous Dirichlet value u0 or Robin ambient u_inf): the source that
// the face fluxes w (x_a - u_face) put on the right-hand side, A x = q + g.
__global__ void boundary_source_kernel(int nx, int ny, int nz, FaceSpec fs, const double *__restrict__ k, double u0,
                                       double u1, double u2, double u3, double u4, double u5, double *__restrict__ g)
{
    const int64_t plane = static_cast<int64_t>(nx) * ny;
    const int64_t n = plane * nz;
    const int64_t a = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const int idx[3] = {static_cast<int>(a % nx), static_cast<int>((a / nx) % ny), static_cast<int>(a / plane)};
    const int dims[3] = {nx, ny, nz};
    const double uf[6] = {u0, u1, u2, u3, u4, u5};
    const double ka = k[a];
    double v = 0.0;
    for (int ax = 0; ax < 3; ++ax) {
        if (idx[ax] == 0) v += face_boundary(fs.bc[2 * ax], ka, fs.d[ax], fs.h[2 * ax]) * uf[2 * ax];
        if (idx[ax] == dims[ax] - 1)
            v += face_boundary(fs.bc[2 * ax + 1], ka, fs.d[ax], fs.h[2 * ax + 1]) * uf[2 * ax + 1];
    }
    g[a] = v;
}

// F[:, j] += alpha g for j < m
__global__ void add_column_kernel(int64_t n, int m, double *__restrict__ F, int64_t ldf, const double *__restrict__ g,
                                  double alpha)
{
    const int64_t a = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const double v = alpha * g[a];
    for (int j = blockIdx.y; j < m; j += gridDim.y) F[static_cast<int64_t>(j) * ldf + a] += v;
}

__global__ void zero_kernel(uint32_t *p, size_t words)
{
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t w = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; w < words; w += stride) p[w] = 0u;
}

// Device copy with 16-byte vector accesses: one vector per thread over a
// grid that covers the buffer (measured on MI355X, a grid of short-lived
// workgroups sustains more bandwidth than fewer workgroups looping over
// several vectors each); a grid-stride loop covers buffers beyond the
// largest grid.  The achievable-bandwidth reference of the HBM-bound kernels.
__global__ __launch_bounds__(256) void copy16_kernel(uint4 *__restrict__ dst, const uint4 *__restrict__ src,
                                                     size_t nvec)
{
    const size_t stride = static_cast<size_t>(gridDim.x) * 256;
    for (size_t e = static_cast<size_t>(blockIdx.x) * 256 + threadIdx.x; e < nvec; e += stride) dst[e] = src[e];
}

bko_status launch_copy16(void *dst, const void *src, size_t bytes, hipStream_t stream)
{
    if (bytes == 0) return BKO_OK;
    const size_t nvec = bytes / 16;
    // grid x workgroup size stays below 2^32 threads
    const size_t blocks = std::min<size_t>((nvec + 255) / 256, (size_t(1) << 23));
    hipLaunchKernelGGL(copy16_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                       static_cast<uint4 *>(dst), static_cast<const uint4 *>(src), nvec);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

bko_status launch_zero(void *p, size_t bytes, hipStream_t stream)
{
    if (bytes == 0) return BKO_OK;
    if ((bytes % 4) != 0 || (reinterpret_cast<uintptr_t>(p) % 4) != 0) {
        set_error("launch_zero: %zu bytes at %p not word aligned", bytes, p);
        return BKO_EINVAL;
    }
    const size_t words = bytes / 4;
    const size_t blocks = std::min<size_t>((words + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                       static_cast<uint32_t *>(p), words);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
}

}  // namespace bko

using namespace bko;

// ------------------------------------------------------------------ C ABI

#define BKO_GUARD_BEGIN try {
#define BKO_GUARD_END                                                     \
    }                                                                     \
    catch (const std::bad_alloc &) {                                      \
        set_error("host allocation failed");                              \
        return BKO_ENOMEM;                                                \
    }                                                                     \
    catch (...) {                                                         \
        set_error("unexpected C++ exception");                            \
        return BKO_EINVAL;                                                \
    }

extern "C" {

const char *bko_version(void) { return "blockoa 0.1 gfx950"; }

const char *bko_last_error(void) { return g_err; }

bko_status bko_operator_bytes(int nx, int ny, int nz, size_t *bytes)
{
    BKO_CHECK(nx >= 1 && ny >= 1 && nz >= 1, "grid %dx%dx%d must be positive", nx, ny, nz);
    BKO_CHECK(bytes != nullptr, "bytes is NULL");
    const int64_t n = static_cast<int64_t>(nx) * ny * nz;
    BKO_CHECK(n <= (int64_t(1) << 31) - 1, "grid of %lld cells exceeds 2^31-1", (long long)n);
    *bytes = coeff_layout(n).bytes;
    return BKO_OK;
}

bko_status bko_assemble_heat_operator(int nx, int ny, int nz, double lx, double ly, double lz,
                                      const double *k_cell_dev, const int bc[6], const double h[6],
                                      void *coeff_dev, size_t coeff_bytes, void *stream,
                                      bko_op *out)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(out != nullptr, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    bko_status st = bko_operator_bytes(nx, ny, nz, &need);
    if (st != BKO_OK) return st;
    BKO_CHECK(std::isfinite(lx) && std::isfinite(ly) && std::isfinite(lz) && lx > 0 && ly > 0 && lz > 0,
              "extents must be positive and finite");
    BKO_CHECK(k_cell_dev != nullptr && coeff_dev != nullptr && bc != nullptr && h != nullptr,
              "NULL pointer argument");
    BKO_CHECK(coeff_bytes >= need, "coefficient buffer has %zu bytes, need %zu", coeff_bytes, need);
    BKO_CHECK(reinterpret_cast<uintptr_t>(coeff_dev) % 256 == 0, "coefficient buffer must be 256-byte aligned");
    bool any_sink = false;
    FaceSpec fs{};
    for (int f = 0; f < 6; ++f) {
        BKO_CHECK(bc[f] == BKO_BC_DIRICHLET0 || bc[f] == BKO_BC_ADIABATIC || bc[f] == BKO_BC_ROBIN,
                  "face %d has unknown kind %d", f, bc[f]);
        if (bc[f] == BKO_BC_ROBIN)
            BKO_CHECK(h[f] > 0.0 && std::isfinite(h[f]), "Robin face %d needs h > 0 (got %g)", f, h[f]);
        any_sink = any_sink || bc[f] != BKO_BC_ADIABATIC;
        fs.bc[f] = bc[f];
        fs.h[f] = bc[f] == BKO_BC_ROBIN ? h[f] : 1.0;
    }
    BKO_CHECK(any_sink, "every face is adiabatic: the operator is singular");
    fs.d[0] = lx / nx;
    fs.d[1] = ly / ny;
    fs.d[2] = lz / nz;
    const int64_t n = static_cast<int64_t>(nx) * ny * nz;
    const CoeffLayout L = coeff_layout(n);
    char *base = static_cast<char *>(coeff_dev);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int *bad = reinterpret_cast<int *>(base + L.status_off);
    st = launch_zero(bad, 256, s);
    if (st != BKO_OK) return st;
    const unsigned blocks = static_cast<unsigned>((n + 255) / 256);
    hipLaunchKernelGGL(assemble_kernel, dim3(blocks), dim3(256), 0, s, nx, ny, nz, fs, k_cell_dev,
                       reinterpret_cast<double *>(base + L.off[0]), reinterpret_cast<double *>(base + L.off[1]),
                       reinterpret_cast<double *>(base + L.off[2]), reinterpret_cast<double *>(base + L.off[3]),
                       reinterpret_cast<float *>(base + L.off[4]), reinterpret_cast<float *>(base + L.off[5]),
                       reinterpret_cast<float *>(base + L.off[6]), reinterpret_cast<float *>(base + L.off[7]), bad);
    BKO_HIP(hipGetLastError());
    int nbad = 0;
    BKO_HIP(hipMemcpyAsync(&nbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    BKO_HIP(hipStreamSynchronize(s));
    if (nbad != 0) {
        set_error("%d cells have conductivity <= 0 or not finite", nbad);
        return BKO_ENOTSPD;
    }
    // every diagonal is positive here (each cell couples to a neighbour or a
    // non-adiabatic face with positive weight), so S is defined
    hipLaunchKernelGGL(scale_coeff_kernel, dim3(blocks), dim3(256), 0, s, nx, ny, nz,
                       reinterpret_cast<const double *>(base + L.off[0]), reinterpret_cast<const double *>(base + L.off[1]),
                       reinterpret_cast<const double *>(base + L.off[2]), reinterpret_cast<const double *>(base + L.off[3]),
                       reinterpret_cast<double *>(base + L.off[8]), reinterpret_cast<double *>(base + L.off[9]),
                       reinterpret_cast<double *>(base + L.off[10]), reinterpret_cast<double *>(base + L.off[11]),
                       reinterpret_cast<float *>(base + L.off[12]), reinterpret_cast<float *>(base + L.off[13]),
                       reinterpret_cast<float *>(base + L.off[14]), reinterpret_cast<float *>(base + L.off[15]),
                       reinterpret_cast<double *>(base + L.off[16]));
    BKO_HIP(hipGetLastError());
    BKO_HIP(hipStreamSynchronize(s));
    Operator *op = new Operator();
    op->nx = nx;
    op->ny = ny;
    op->nz = nz;
    op->lx = lx;
    op->ly = ly;
    op->lz = lz;
    op->n = n;
    op->coeff = coeff_dev;
    op->diag64 = reinterpret_cast<const double *>(base + L.off[0]);
    op->wx64 = reinterpret_cast<const double *>(base + L.off[1]);
    op->wy64 = reinterpret_cast<const double *>(base + L.off[2]);
    op->wz64 = reinterpret_cast<const double *>(base + L.off[3]);
    op->diag32 = reinterpret_cast<const float *>(base + L.off[4]);
    op->wx32 = reinterpret_cast<const float *>(base + L.off[5]);
    op->wy32 = reinterpret_cast<const float *>(base + L.off[6]);
    op->wz32 = reinterpret_cast<const float *>(base + L.off[7]);
    op->sdiag64 = reinterpret_cast<const double *>(base + L.off[8]);
    op->swx64 = reinterpret_cast<const double *>(base + L.off[9]);
    op->swy64 = reinterpret_cast<const double *>(base + L.off[10]);
    op->swz64 = reinterpret_cast<const double *>(base + L.off[11]);
    op->sdiag32 = reinterpret_cast<const float *>(base + L.off[12]);
    op->swx32 = reinterpret_cast<const float *>(base + L.off[13]);
    op->swy32 = reinterpret_cast<const float *>(base + L.off[14]);
    op->swz32 = reinterpret_cast<const float *>(base + L.off[15]);
    op->scale64 = reinterpret_cast<const double *>(base + L.off[16]);
    op->precond = BKO_PRECOND_NONE;
    for (int f = 0; f < 6; ++f) {
        op->bc[f] = fs.bc[f];
        op->h[f] = fs.h[f];
    }
    *out = reinterpret_cast<bko_op>(op);
    return BKO_OK;
    BKO_GUARD_END
}

bko_status bko_operator_dims(bko_op A, int *nx, int *ny, int *nz)
{
    BKO_CHECK(A != nullptr, "operator handle is NULL");
    const Operator *op = reinterpret_cast<const Operator *>(A);
    if (nx) *nx = op->nx;
    if (ny) *ny = op->ny;
    if (nz) *nz = op->nz;
    return BKO_OK;
}

bko_status bko_operator_set_precond(bko_op A, int kind)
{
    BKO_CHECK(A != nullptr, "operator handle is NULL");
    BKO_CHECK(kind == BKO_PRECOND_NONE || kind == BKO_PRECOND_JACOBI, "unknown preconditioner %d", kind);
    reinterpret_cast<Operator *>(A)->precond = kind;
    return BKO_OK;
}

bko_status bko_operator_get_precond(bko_op A, int *kind)
{
    BKO_CHECK(A != nullptr && kind != nullptr, "NULL argument");
    *kind = reinterpret_cast<const Operator *>(A)->precond;
    return BKO_OK;
}

bko_status bko_boundary_source(bko_op A, const double *k_cell_dev, const double u_face[6], double *g, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(A != nullptr && k_cell_dev != nullptr && u_face != nullptr && g != nullptr, "NULL argument");
    const Operator &op = *reinterpret_cast<const Operator *>(A);
    for (int f = 0; f < 6; ++f) BKO_CHECK(std::isfinite(u_face[f]), "face value %d is not finite", f);
    FaceSpec fs{};
    for (int f = 0; f < 6; ++f) {
        fs.bc[f] = op.bc[f];
        fs.h[f] = op.h[f];
    }
    fs.d[0] = op.lx / op.nx;
    fs.d[1] = op.ly / op.ny;
    fs.d[2] = op.lz / op.nz;
    const unsigned blocks = static_cast<unsigned>((op.n + 255) / 256);
    hipLaunchKernelGGL(boundary_source_kernel, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream), op.nx,
                       op.ny, op.nz, fs, k_cell_dev, u_face[0], u_face[1], u_face[2], u_face[3], u_face[4], u_face[5], g);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
    BKO_GUARD_END
}

bko_status bko_add_column(int n, int m, double *F, int ldf, const double *g, double alpha, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(n >= 0 && m >= 0, "bad sizes n=%d m=%d", n, m);
    if (n == 0 || m == 0) return BKO_OK;
    BKO_CHECK(F != nullptr && g != nullptr && ldf >= n, "bad arguments");
    const dim3 grid(static_cast<unsigned>((n + 255) / 256), static_cast<unsigned>(std::min(m, 256)));
    hipLaunchKernelGGL(add_column_kernel, grid, dim3(256), 0, static_cast<hipStream_t>(stream), static_cast<int64_t>(n), m,
                       F, static_cast<int64_t>(ldf), g, alpha);
    BKO_HIP(hipGetLastError());
    return BKO_OK;
    BKO_GUARD_END
}

bko_status bko_destroy_operator(bko_op A)
{
    delete reinterpret_cast<Operator *>(A);
    return BKO_OK;
}

static bool valid_dtype(int t) { return t == BKO_F64 || t == BKO_F32 || t == BKO_BF16; }

bko_status bko_apply_operator(bko_op A, int m, const void *T, int ldt, bko_dtype t_t, void *F, int ldf,
                              bko_dtype f_t, bko_dtype compute, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(A != nullptr, "operator handle is NULL");
    const Operator &op = *reinterpret_cast<const Operator *>(A);
    BKO_CHECK(m >= 0, "m = %d < 0", m);
    BKO_CHECK(valid_dtype(t_t) && valid_dtype(f_t) && valid_dtype(compute), "bad dtype");
    if (m == 0) return BKO_OK;
    BKO_CHECK(T != nullptr && F != nullptr, "NULL array");
    BKO_CHECK(ldt >= op.n && ldf >= op.n, "leading dimensions (%d, %d) must be >= n = %lld", ldt, ldf,
              (long long)op.n);
    const char *t0 = static_cast<const char *>(T);
    const char *t1 = t0 + dtype_size(t_t) * (static_cast<size_t>(ldt) * (m - 1) + op.n);
    const char *f0 = static_cast<const char *>(F);
    const char *f1 = f0 + dtype_size(f_t) * (static_cast<size_t>(ldf) * (m - 1) + op.n);
    BKO_CHECK(t1 <= f0 || f1 <= t0, "T and F overlap");
    TimedLaunch tl(kApply, static_cast<hipStream_t>(stream));
    return launch_stencil(op, m, T, ldt, t_t, F, ldf, f_t, compute, nullptr, 0,
                          static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

bko_status bko_copy(void *dst, const void *src, size_t bytes, void *stream)
{
    BKO_GUARD_BEGIN
    if (bytes == 0) return BKO_OK;
    BKO_CHECK(dst != nullptr && src != nullptr, "NULL array");
    BKO_CHECK(bytes % 16 == 0 && reinterpret_cast<uintptr_t>(dst) % 16 == 0 &&
                  reinterpret_cast<uintptr_t>(src) % 16 == 0,
              "copy of %zu bytes needs 16-byte aligned pointers and a multiple of 16 bytes", bytes);
    const char *s0 = static_cast<const char *>(src), *d0 = static_cast<const char *>(dst);
    BKO_CHECK(s0 + bytes <= d0 || d0 + bytes <= s0, "source and destination overlap");
    return launch_copy16(dst, src, bytes, static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

bko_status bko_apply_operator_tiling(bko_op A, int m, const void *T, int ldt, bko_dtype t_t, const void *F, int ldf,
                                     bko_dtype f_t, bko_dtype compute, int *tile_rows)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(A != nullptr && tile_rows != nullptr, "NULL argument");
    const Operator &op = *reinterpret_cast<const Operator *>(A);
    BKO_CHECK(m >= 0 && ldt >= op.n && ldf >= op.n, "bad sizes");
    BKO_CHECK(valid_dtype(t_t) && valid_dtype(f_t) && valid_dtype(compute), "bad dtype");
    *tile_rows = stencil_tile_rows(op, m, T, ldt, t_t, F, ldf, f_t, compute);
    return BKO_OK;
    BKO_GUARD_END
}

bko_status bko_residual(bko_op A, int m, const double *B, int ldb, const double *X, int ldx, double *R,
                        int ldr, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(A != nullptr, "operator handle is NULL");
    const Operator &op = *reinterpret_cast<const Operator *>(A);
    BKO_CHECK(m >= 0, "m = %d < 0", m);
    if (m == 0) return BKO_OK;
    BKO_CHECK(B && X && R, "NULL array");
    BKO_CHECK(ldb >= op.n && ldx >= op.n && ldr >= op.n, "leading dimensions must be >= n");
    BKO_CHECK(!(R == B && ldr != ldb), "R aliases B with a different leading dimension");
    TimedLaunch tl(kResid, static_cast<hipStream_t>(stream));
    return launch_stencil(op, m, X, ldx, BKO_F64, R, ldr, BKO_F64, BKO_F64, B, ldb,
                          static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

bko_status bko_combine(int n, int s, int m, const void *X, int ldx, bko_dtype x_t, const void *C, int ldc,
                       bko_dtype c_t, void *T, int ldt, bko_dtype t_t, bko_dtype compute, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(n >= 0 && s >= 1 && m >= 0, "bad sizes n=%d s=%d m=%d", n, s, m);
    BKO_CHECK(s <= 64, "s = %d exceeds the supported maximum of 64", s);
    BKO_CHECK(valid_dtype(x_t) && valid_dtype(c_t) && valid_dtype(t_t) && valid_dtype(compute), "bad dtype");
    if (n == 0 || m == 0) return BKO_OK;
    BKO_CHECK(X && C && T, "NULL array");
    BKO_CHECK(ldx >= n && ldc >= s && ldt >= n, "bad leading dimension");
    TimedLaunch tl(kCombine, static_cast<hipStream_t>(stream));
    return launch_combine(n, s, m, X, ldx, x_t, C, ldc, c_t, T, ldt, t_t, compute,
                          static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

static bool noise_ok(const bko_noise *nz)
{
    return nz == nullptr || ((nz->kind == BKO_NOISE_NONE || nz->kind == BKO_NOISE_UNIFORM ||
                              nz->kind == BKO_NOISE_GAUSSIAN) && std::isfinite(nz->amplitude) && nz->amplitude >= 0.0);
}

bko_status bko_combine_noisy(int n, int s, int m, const double *X, int ldx, const double *C, int ldc, double *T,
                             int ldt, const bko_noise *noise, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(n >= 0 && s >= 1 && s <= 64 && m >= 0, "bad sizes n=%d s=%d m=%d", n, s, m);
    BKO_CHECK(noise_ok(noise), "bad noise description");
    if (n == 0 || m == 0) return BKO_OK;
    BKO_CHECK(X && C && T, "NULL array");
    BKO_CHECK(ldx >= n && ldc >= s && ldt >= n, "bad leading dimension");
    const int kind = noise ? noise->kind : BKO_NOISE_NONE;
    TimedLaunch tl(kCombine, static_cast<hipStream_t>(stream));
    return launch_combine_noisy(n, s, m, X, ldx, C, ldc, T, ldt, kind, noise ? noise->amplitude : 0.0,
                                noise ? noise->seed : 0, noise ? noise->field_offset : 0, static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

bko_status bko_noise_fill(int n, int m, double *E, int lde, const bko_noise *noise, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(n >= 0 && m >= 0 && m <= 65535, "bad sizes n=%d m=%d (m <= 65535 per call)", n, m);
    BKO_CHECK(noise != nullptr && noise_ok(noise), "bad noise description");
    if (n == 0 || m == 0) return BKO_OK;
    BKO_CHECK(E != nullptr && lde >= n, "bad output");
    return launch_noise_fill(n, m, E, lde, noise->kind, noise->amplitude, noise->seed, noise->field_offset,
                             static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

bko_status bko_normalize_weights(int s, int m, double *C, int ldc, double min_abs_sum, int *flags, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(s >= 1 && m >= 0 && ldc >= s, "bad sizes s=%d m=%d ldc=%d", s, m, ldc);
    BKO_CHECK(std::isfinite(min_abs_sum) && min_abs_sum >= 0.0, "min_abs_sum must be finite and >= 0");
    if (m == 0) return BKO_OK;
    BKO_CHECK(C != nullptr && flags != nullptr, "NULL argument");
    return launch_normalize_weights(s, m, C, ldc, min_abs_sum, flags, static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

static int64_t combine_apply_ld(int64_t n) { return static_cast<int64_t>(align_up(static_cast<size_t>(n), 32)); }

bko_status bko_combine_apply_workspace_bytes(bko_op A, int s, size_t *bytes)
{
    BKO_CHECK(A != nullptr && bytes != nullptr, "NULL argument");
    BKO_CHECK(s >= 1 && s <= 64, "s = %d outside [1, 64]", s);
    const Operator *op = reinterpret_cast<const Operator *>(A);
    *bytes = sizeof(double) * static_cast<size_t>(combine_apply_ld(op->n)) * s;
    return BKO_OK;
}

bko_status bko_combine_apply(bko_op A, int s, int m, const double *X, int ldx, const double *C, int ldc, double *T,
                             int ldt, double *F, int ldf, void *work, size_t work_bytes, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(A != nullptr, "operator handle is NULL");
    const Operator &op = *reinterpret_cast<const Operator *>(A);
    const int64_t n = op.n;
    BKO_CHECK(s >= 1 && s <= 64 && m >= 0, "bad sizes s=%d m=%d", s, m);
    if (m == 0) return BKO_OK;
    BKO_CHECK(X && C && T && F, "NULL array");
    BKO_CHECK(ldx >= n && ldc >= s && ldt >= n && ldf >= n, "bad leading dimension");
    size_t need = 0;
    bko_status st = bko_combine_apply_workspace_bytes(A, s, &need);
    if (st != BKO_OK) return st;
    BKO_CHECK(work != nullptr && work_bytes >= need, "workspace has %zu bytes, need %zu", work_bytes, need);
    BKO_CHECK(reinterpret_cast<uintptr_t>(work) % 256 == 0, "workspace must be 256-byte aligned");
    hipStream_t sm = static_cast<hipStream_t>(stream);
    double *Y = static_cast<double *>(work);
    const int64_t ldy = combine_apply_ld(n);
    // Y = A X for the s basis columns, then T = X C and F = Y C in one pass
    if ((st = launch_stencil(op, s, X, ldx, BKO_F64, Y, ldy, BKO_F64, BKO_F64, nullptr, 0, sm)) != BKO_OK) return st;
    TimedLaunch tl(kCombine, sm);
    return launch_combine_dual(n, s, m, X, ldx, Y, ldy, C, ldc, T, ldt, F, ldf, sm);
    BKO_GUARD_END
}

bko_status bko_block_krylov_workspace_bytes(bko_op A, int s, bko_dtype compute, size_t *bytes)
{
    BKO_CHECK(A != nullptr && bytes != nullptr, "NULL argument");
    BKO_CHECK(s >= 1 && s <= 64, "s = %d outside [1, 64]", s);
    BKO_CHECK(compute == BKO_F64 || compute == BKO_F32, "compute must be BKO_F64 or BKO_F32");
    *bytes = solve_workspace_bytes(reinterpret_cast<const Operator *>(A)->n, s, compute);
    return BKO_OK;
}

bko_status bko_block_krylov_solve(bko_op A, int s, const double *B, int ldb, double *X, int ldx,
                                  const double *X0, int ldx0, bko_dtype compute, double tol, int max_iter,
                                  void *work, size_t work_bytes, bko_solve_info *info, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(A != nullptr, "operator handle is NULL");
    const Operator &op = *reinterpret_cast<const Operator *>(A);
    BKO_CHECK(s >= 1 && s <= 64, "s = %d outside [1, 64]", s);
    BKO_CHECK(compute == BKO_F64 || compute == BKO_F32, "compute must be BKO_F64 or BKO_F32");
    BKO_CHECK(B && X && work, "NULL array");
    BKO_CHECK(ldb >= op.n && ldx >= op.n, "leading dimensions must be >= n");
    BKO_CHECK(X0 == nullptr || ldx0 >= op.n, "ldx0 must be >= n");
    BKO_CHECK(tol > 0.0 && std::isfinite(tol), "tol must be positive");
    BKO_CHECK(max_iter >= 1, "max_iter must be >= 1");
    BKO_CHECK(reinterpret_cast<uintptr_t>(work) % 256 == 0, "workspace must be 256-byte aligned");
    const size_t need = solve_workspace_bytes(op.n, s, compute);
    if (work_bytes < need) {
        set_error("workspace has %zu bytes, need %zu", work_bytes, need);
        return BKO_ENOMEM;
    }
    if (X0 == X) BKO_CHECK(ldx0 == ldx, "X0 aliases X with a different leading dimension");
    return block_solve(op, s, B, ldb, X, ldx, X0, ldx0, compute, tol, max_iter, work, work_bytes, info,
                       static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

bko_status bko_cg_workspace_bytes(bko_op A, int m, size_t *bytes)
{
    BKO_CHECK(A != nullptr && bytes != nullptr, "NULL argument");
    BKO_CHECK(m >= 1 && m <= 65535, "m = %d outside [1, 65535]", m);
    *bytes = cg_workspace_bytes(reinterpret_cast<const Operator *>(A)->n, m);
    return BKO_OK;
}

bko_status bko_cg_solve(bko_op A, int m, const double *B, int ldb, double *X, int ldx, double tol, int max_iter,
                        void *work, size_t work_bytes, int *iters, bko_solve_info *info, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(A != nullptr, "operator handle is NULL");
    const Operator &op = *reinterpret_cast<const Operator *>(A);
    BKO_CHECK(m >= 1 && m <= 65535, "m = %d outside [1, 65535]", m);
    BKO_CHECK(B && X && work, "NULL array");
    BKO_CHECK(ldb >= op.n && ldx >= op.n, "leading dimensions must be >= n");
    BKO_CHECK(tol > 0.0 && std::isfinite(tol), "tol must be positive");
    BKO_CHECK(max_iter >= 1, "max_iter must be >= 1");
    BKO_CHECK(reinterpret_cast<uintptr_t>(work) % 256 == 0, "workspace must be 256-byte aligned");
    const size_t need = cg_workspace_bytes(op.n, m);
    if (work_bytes < need) {
        set_error("workspace has %zu bytes, need %zu", work_bytes, need);
        return BKO_ENOMEM;
    }
    return cg_solve(op, m, B, ldb, X, ldx, tol, max_iter, work, iters, info, static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

bko_status bko_batch_plan_create(int nchips, const bko_op *ops, int s, const int *m, const bko_dtype dt[4],
                                 bko_batch *out)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(out != nullptr && ops != nullptr && dt != nullptr, "NULL argument");
    *out = nullptr;
    BKO_CHECK(nchips >= 1 && nchips <= 65535, "nchips = %d outside [1, 65535]", nchips);
    BKO_CHECK(s >= 1 && s <= 64, "s = %d outside [1, 64]", s);
    BKO_CHECK(dt[0] == BKO_F64 || dt[0] == BKO_F32, "dt[0] (block iteration) must be BKO_F64 or BKO_F32");
    BKO_CHECK(valid_dtype(dt[1]) && valid_dtype(dt[2]) && valid_dtype(dt[3]), "bad output dtype");
    for (int c = 0; c < nchips; ++c) BKO_CHECK(ops[c] != nullptr, "operator %d is NULL", c);
    if (m)
        for (int c = 0; c < nchips; ++c) BKO_CHECK(m[c] >= 0, "m of chip %d is negative", c);
    BatchPlan *p = new BatchPlan();
    p->s = s;
    p->compute = dt[0];
    p->comb_compute = dt[1];
    p->t_dtype = dt[2];
    p->f_dtype = dt[3];
    p->apply_compute = (dt[2] == BKO_F64 && dt[3] == BKO_F64) ? BKO_F64 : BKO_F32;
    for (int c = 0; c < nchips; ++c) p->ops.push_back(reinterpret_cast<const Operator *>(ops[c]));
    if (m) p->m.assign(m, m + nchips);
    *out = reinterpret_cast<bko_batch>(p);
    return BKO_OK;
    BKO_GUARD_END
}

bko_status bko_batch_plan_destroy(bko_batch plan)
{
    delete reinterpret_cast<BatchPlan *>(plan);
    return BKO_OK;
}

bko_status bko_batch_workspace_bytes(bko_batch plan, size_t *bytes)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(plan != nullptr && bytes != nullptr, "NULL argument");
    *bytes = batch_workspace_bytes(*reinterpret_cast<BatchPlan *>(plan));
    return BKO_OK;
    BKO_GUARD_END
}

static bko_status check_batch_work(const BatchPlan &p, void *work, size_t work_bytes)
{
    BKO_CHECK(work != nullptr, "NULL workspace");
    BKO_CHECK(reinterpret_cast<uintptr_t>(work) % 256 == 0, "workspace must be 256-byte aligned");
    const size_t need = batch_workspace_bytes(p);
    if (work_bytes < need) {
        set_error("workspace has %zu bytes, need %zu", work_bytes, need);
        return BKO_ENOMEM;
    }
    return BKO_OK;
}

bko_status bko_batch_tune(bko_batch plan, void *work, size_t work_bytes, int *tiles_per_wg, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(plan != nullptr, "NULL plan");
    BatchPlan &p = *reinterpret_cast<BatchPlan *>(plan);
    bko_status rc = check_batch_work(p, work, work_bytes);
    if (rc != BKO_OK) return rc;
    rc = batch_tune(p, work, static_cast<hipStream_t>(stream));
    if (rc == BKO_OK && tiles_per_wg) *tiles_per_wg = p.tiles_per_wg;
    return rc;
    BKO_GUARD_END
}

bko_status bko_batch_solve(bko_batch plan, const double *const *B, const int *ldb, double *const *X, const int *ldx,
                           const double *const *X0, const int *ldx0, double tol, int max_iter, void *work,
                           size_t work_bytes, bko_solve_info *infos, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(plan != nullptr, "NULL plan");
    BatchPlan &p = *reinterpret_cast<BatchPlan *>(plan);
    const int nc = static_cast<int>(p.ops.size());
    BKO_CHECK(B && ldb && X && ldx, "NULL array table");
    BKO_CHECK(X0 == nullptr || ldx0 != nullptr, "X0 given without ldx0");
    BKO_CHECK(tol > 0.0 && std::isfinite(tol), "tol must be positive");
    BKO_CHECK(max_iter >= 1, "max_iter must be >= 1");
    std::vector<int64_t> lb(nc), lx(nc), lx0(nc, 0);
    for (int c = 0; c < nc; ++c) {
        const int64_t n = p.ops[c]->n;
        BKO_CHECK(B[c] && X[c], "NULL array of chip %d", c);
        BKO_CHECK(ldb[c] >= n && ldx[c] >= n, "leading dimensions of chip %d must be >= n", c);
        lb[c] = ldb[c];
        lx[c] = ldx[c];
        if (X0 && X0[c]) {
            BKO_CHECK(ldx0[c] >= n, "ldx0 of chip %d must be >= n", c);
            if (X0[c] == X[c]) BKO_CHECK(ldx0[c] == ldx[c], "X0 of chip %d aliases X with another ld", c);
            lx0[c] = ldx0[c];
        }
    }
    bko_status rc = check_batch_work(p, work, work_bytes);
    if (rc != BKO_OK) return rc;
    return batch_solve(p, B, lb.data(), X, lx.data(), X0, lx0.data(), tol, max_iter, work, infos,
                       static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

}  // extern "C"

// Output knobs chosen by timing, per device architecture and batch shape
// bucket (chips, total cells to a power of two, largest field count, s and
// the dtypes), shared by every plan of the process.
static std::mutex g_out_tune_mu;
static std::map<std::string, std::pair<int, int64_t>> g_out_tune_cache;

static std::string out_tune_key(const BatchPlan &p)
{
    hipDeviceProp_t prop{};
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) arch = prop.gcnArchName;
    int64_t cells = 0;
    int mmax = 0;
    for (size_t c = 0; c < p.ops.size(); ++c) {
        cells += p.ops[c]->n;
        mmax = std::max(mmax, p.m[c]);
    }
    int lg = 0;
    while ((int64_t(1) << lg) < cells) ++lg;
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s|%zu|%d|%d|%d|%d%d%d", arch.c_str(), p.ops.size(), lg, mmax, p.s,
                  static_cast<int>(p.comb_compute), static_cast<int>(p.t_dtype), static_cast<int>(p.f_dtype));
    return buf;
}

namespace {

struct OutArgs {
    std::vector<int64_t> n, lx, lc, lt, lf;
    const double *const *X;
    const double *const *C;
    void *const *T;
    void *const *F;
    void *sjobs, *cjobs;
    std::vector<unsigned char> hs, hc;  // host job tables, alive until the stream has passed the launches
};

bko_status out_combine(BatchPlan &p, OutArgs &a, int64_t fpw, hipStream_t st)
{
    return launch_combine_group(static_cast<int>(p.ops.size()), a.n.data(), p.s, p.m.data(), a.X, a.lx.data(), a.C,
                                a.lc.data(), a.T, a.lt.data(), p.t_dtype, p.comb_compute, fpw, a.cjobs, a.hc, st);
}

bko_status out_apply(BatchPlan &p, OutArgs &a, int ty_cap, hipStream_t st)
{
    return launch_stencil_group(p.ops.data(), static_cast<int>(p.ops.size()), p.m.data(),
                                reinterpret_cast<const void *const *>(a.T), a.lt.data(), p.t_dtype, a.F, a.lf.data(),
                                p.f_dtype, p.apply_compute, ty_cap, a.sjobs, a.hs, st);
}

// Milliseconds of one launch of fn (after one untimed launch).
template <class Fn>
bko_status time_once(Fn fn, hipStream_t st, float &ms)
{
    bko_status rc = fn();
    if (rc != BKO_OK) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BKO_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(hipErrorOutOfMemory, "hipEventCreate");
    }
    bool ok = hipEventRecord(e0, st) == hipSuccess;
    rc = fn();
    ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
         hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != BKO_OK) return rc;
    if (!ok) return hip_fail(hipErrorUnknown, "output timing events");
    return BKO_OK;
}

// First run of a plan: the tile height cap of the grouped operator action
// and the fields per workgroup of the grouped combination, each picked
// from a few candidates by timing them on the call's own outputs (every
// candidate writes the same T and F).
bko_status tune_outputs(BatchPlan &p, OutArgs &a, hipStream_t st)
{
    const std::string key = out_tune_key(p);
    {
        std::lock_guard<std::mutex> lock(g_out_tune_mu);
        auto it = g_out_tune_cache.find(key);
        if (it != g_out_tune_cache.end()) {
            p.out_ty_cap = it->second.first;
            p.out_fields_per_wg = it->second.second;
            p.out_tuned = true;
            return BKO_OK;
        }
    }
    p.out_tune_ms.clear();
    bko_status rc;
    float best = 0.f;
    int64_t best_fpw = 0;
    for (int64_t fpw : {int64_t(0), int64_t(64), int64_t(256)}) {
        float ms = 0.f;
        if ((rc = time_once([&] { return out_combine(p, a, fpw, st); }, st, ms)) != BKO_OK) return rc;
        p.out_tune_ms.emplace_back("fields_per_wg=" + std::to_string(fpw), ms);
        if (fpw == 0 || ms < best) best = ms, best_fpw = fpw;
    }
    int best_ty = 0;
    for (int ty : {0, 16, 8}) {
        float ms = 0.f;
        if ((rc = time_once([&] { return out_apply(p, a, ty, st); }, st, ms)) != BKO_OK) return rc;
        p.out_tune_ms.emplace_back("tile_rows_cap=" + std::to_string(ty), ms);
        if (ty == 0 || ms < best) best = ms, best_ty = ty;
    }
    p.out_ty_cap = best_ty;
    p.out_fields_per_wg = best_fpw;
    p.out_tuned = true;
    std::lock_guard<std::mutex> lock(g_out_tune_mu);
    g_out_tune_cache[key] = {best_ty, best_fpw};
    return BKO_OK;
}

}  // namespace

extern "C" {

bko_status bko_batch_run(bko_batch plan, const double *const *B, const int *ldb, double *const *X, const int *ldx,
                         const double *const *C, const int *ldc, void *const *T, const int *ldt, void *const *F,
                         const int *ldf, double tol, int max_iter, void *work, size_t work_bytes,
                         bko_solve_info *infos, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(plan != nullptr, "NULL plan");
    BatchPlan &p = *reinterpret_cast<BatchPlan *>(plan);
    const int nc = static_cast<int>(p.ops.size());
    BKO_CHECK(!p.m.empty(), "the plan was created without field counts (m = NULL): use bko_batch_solve");
    BKO_CHECK(B && ldb && X && ldx && C && ldc && T && ldt && F && ldf, "NULL array table");
    BKO_CHECK(tol > 0.0 && std::isfinite(tol), "tol must be positive");
    BKO_CHECK(max_iter >= 1, "max_iter must be >= 1");
    OutArgs a;
    a.n.resize(nc);
    a.lx.resize(nc);
    a.lc.resize(nc);
    a.lt.resize(nc);
    a.lf.resize(nc);
    std::vector<int64_t> lb(nc), lx0(nc, 0);
    const size_t wt = dtype_size(p.t_dtype), wf = dtype_size(p.f_dtype);
    for (int c = 0; c < nc; ++c) {
        const int64_t n = p.ops[c]->n;
        const int mc = p.m[c];
        BKO_CHECK(B[c] && X[c], "NULL array of chip %d", c);
        BKO_CHECK(ldb[c] >= n && ldx[c] >= n, "leading dimensions of chip %d must be >= n", c);
        if (mc > 0) {
            BKO_CHECK(C[c] && T[c] && F[c], "NULL output array of chip %d", c);
            BKO_CHECK(ldc[c] >= p.s && ldt[c] >= n && ldf[c] >= n, "output leading dimensions of chip %d", c);
            const char *t0 = static_cast<const char *>(T[c]), *f0 = static_cast<const char *>(F[c]);
            const char *t1 = t0 + wt * (static_cast<size_t>(ldt[c]) * (mc - 1) + n);
            const char *f1 = f0 + wf * (static_cast<size_t>(ldf[c]) * (mc - 1) + n);
            BKO_CHECK(t1 <= f0 || f1 <= t0, "T and F of chip %d overlap", c);
        }
        a.n[c] = n;
        lb[c] = ldb[c];
        a.lx[c] = ldx[c];
        a.lc[c] = ldc[c];
        a.lt[c] = ldt[c];
        a.lf[c] = ldf[c];
    }
    bko_status rc = check_batch_work(p, work, work_bytes);
    if (rc != BKO_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // basis solutions of every chip (Sec. III-A, Eq. (4))
    const bko_status solved = batch_solve(p, B, lb.data(), X, a.lx.data(), nullptr, lx0.data(), tol, max_iter, work,
                                          infos, st);
    if (solved != BKO_OK && solved != BKO_ENOCONV && solved != BKO_EBREAKDOWN) return solved;
    // T = X C (Sec. III-B, Eq. (5)) and F = A T (Sec. III-C, Eq. (6)) of
    // every chip: one grouped combination, then one grouped operator action
    // of the T written
    char *tables = static_cast<char *>(work) + batch_solve_bytes(p);
    a.sjobs = tables;
    a.cjobs = tables + align_up(stencil_group_job_bytes(nc), 256);
    a.X = X;
    a.C = C;
    a.T = T;
    a.F = F;
    if (!p.out_tuned && (rc = tune_outputs(p, a, st)) != BKO_OK) return rc;
    {
        TimedLaunch tl(kCombine, st);
        if ((rc = out_combine(p, a, p.out_fields_per_wg, st)) != BKO_OK) return rc;
    }
    {
        TimedLaunch tl(kApply, st);
        if ((rc = out_apply(p, a, p.out_ty_cap, st)) != BKO_OK) return rc;
    }
    BKO_HIP(hipStreamSynchronize(st));
    return solved;  // the solve's message stays the last error when it is not BKO_OK
    BKO_GUARD_END
}

bko_status bko_batch_output_tuning(bko_batch plan, int *tile_rows_cap, int64_t *fields_per_wg)
{
    BKO_CHECK(plan != nullptr, "NULL plan");
    const BatchPlan &p = *reinterpret_cast<const BatchPlan *>(plan);
    if (tile_rows_cap) *tile_rows_cap = p.out_tuned ? p.out_ty_cap : -1;
    if (fields_per_wg) *fields_per_wg = p.out_tuned ? p.out_fields_per_wg : -1;
    return BKO_OK;
}

// ------------------------------------------------------------------ learned start

bko_status bko_nn_conv2d(const float *A, int Ca, const float *B, int Cb, int mode, int N, int H, int W, int Co, int K,
                         const uint16_t *wgt, int transposed, const float *bias, float *out, int relu, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(A && wgt && out, "NULL array");
    BKO_CHECK(N >= 1 && H >= 1 && W >= 1 && Ca >= 1 && Co >= 1, "bad sizes");
    BKO_CHECK(K == 1 || K == 3, "K must be 1 or 3");
    BKO_CHECK(mode >= 0 && mode <= 2, "mode must be 0, 1 or 2");
    BKO_CHECK(mode == 2 ? (B != nullptr && Cb >= 1 && H % 2 == 0 && W % 2 == 0) : Cb == 0, "bad concatenation input");
    return nn_conv(A, Ca, B, Cb, mode, N, H, W, Co, K, wgt, transposed, bias, out, relu,
                   static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

size_t bko_nn_wgrad_work_floats(int N, int H, int W, int Ci, int Co, int K)
{
    if (N < 1 || H < 1 || W < 1 || Ci < 1 || Co < 1 || (K != 1 && K != 3)) return 0;
    return nn_wgrad_part_floats(N, H, W, Ci, Co, K);
}

bko_status bko_nn_conv2d_wgrad(const float *A, int Ca, const float *B, int Cb, int mode, const float *g, int N, int H,
                               int W, int Co, int K, float *work, float *gw, float *gb, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(A && g && work && gw && gb, "NULL array");
    BKO_CHECK(N >= 1 && H >= 1 && W >= 1 && Ca >= 1 && Co >= 1, "bad sizes");
    BKO_CHECK(K == 1 || K == 3, "K must be 1 or 3");
    BKO_CHECK(mode >= 0 && mode <= 2, "mode must be 0, 1 or 2");
    BKO_CHECK(mode == 2 ? (B != nullptr && Cb >= 1 && H % 2 == 0 && W % 2 == 0) : Cb == 0, "bad concatenation input");
    return nn_wgrad(A, Ca, B, Cb, mode, g, N, H, W, Co, K, work, gw, gb, static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

bko_status bko_unet_create(int cin, int cout, int base, int height, int width, int max_batch, bko_net *out)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(out != nullptr, "NULL argument");
    *out = nullptr;
    BKO_CHECK(cin >= 1 && cout >= 1 && base >= 1 && max_batch >= 1, "bad sizes");
    BKO_CHECK(height >= 8 && width >= 8 && height % 8 == 0 && width % 8 == 0,
              "height and width must be positive multiples of 8 (three 2x poolings)");
    *out = reinterpret_cast<bko_net>(new UNet(cin, cout, base, height, width, max_batch));
    return BKO_OK;
    BKO_GUARD_END
}

bko_status bko_unet_destroy(bko_net net)
{
    delete reinterpret_cast<UNet *>(net);
    return BKO_OK;
}

bko_status bko_unet_sizes(bko_net net, int64_t *nparams, size_t *state_bytes, size_t *work_bytes)
{
    BKO_CHECK(net != nullptr, "NULL network");
    const UNet &u = *reinterpret_cast<UNet *>(net);
    if (nparams) *nparams = u.nparams;
    if (state_bytes) *state_bytes = u.state_bytes();
    if (work_bytes) *work_bytes = u.work_floats * sizeof(float);
    return BKO_OK;
}

bko_status bko_unet_set_params(bko_net net, void *state, const float *params, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(net && state && params, "NULL argument");
    BKO_CHECK(reinterpret_cast<uintptr_t>(state) % 256 == 0, "state must be 256-byte aligned");
    return reinterpret_cast<UNet *>(net)->set_params(state, params, static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

bko_status bko_unet_forward(bko_net net, void *state, void *work, const float *x, int n, float *y, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(net && state && work && x && y, "NULL argument");
    const UNet &u = *reinterpret_cast<UNet *>(net);
    BKO_CHECK(n >= 1 && n <= u.batch, "n = %d outside [1, %d]", n, u.batch);
    BKO_CHECK(reinterpret_cast<uintptr_t>(state) % 256 == 0 && reinterpret_cast<uintptr_t>(work) % 256 == 0,
              "state and work must be 256-byte aligned");
    return u.forward(state, work, x, n, y, static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

bko_status bko_unet_infer(bko_net net, void *state, void *work, const float *x, int n, float *y, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(net && state && work && x && y, "NULL argument");
    const UNet &u = *reinterpret_cast<UNet *>(net);
    BKO_CHECK(n >= 1 && n <= u.batch, "n = %d outside [1, %d]", n, u.batch);
    BKO_CHECK(reinterpret_cast<uintptr_t>(state) % 256 == 0 && reinterpret_cast<uintptr_t>(work) % 256 == 0,
              "state and work must be 256-byte aligned");
    return u.forward(state, work, x, n, y, static_cast<hipStream_t>(stream), true);
    BKO_GUARD_END
}

bko_status bko_unet_gradient(bko_net net, void *state, void *work, const float *x, const float *target, int n,
                             float *loss, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(net && state && work && x && target, "NULL argument");
    const UNet &u = *reinterpret_cast<UNet *>(net);
    BKO_CHECK(n >= 1 && n <= u.batch, "n = %d outside [1, %d]", n, u.batch);
    BKO_CHECK(reinterpret_cast<uintptr_t>(state) % 256 == 0 && reinterpret_cast<uintptr_t>(work) % 256 == 0,
              "state and work must be 256-byte aligned");
    return u.gradient(state, work, x, target, n, loss, static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

bko_status bko_unet_adam_step(bko_net net, void *state, float lr, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(net && state, "NULL argument");
    BKO_CHECK(lr > 0.0f && std::isfinite(lr), "lr must be positive");
    return reinterpret_cast<UNet *>(net)->adam(state, lr, static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

bko_status bko_lstart_pack(int nx, int ny, int nz, const double *F, int ldf, int m, const double *k_cell, float kmu,
                           float ksig, float hval, double *scale, float *x, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(F && k_cell && scale && x, "NULL argument");
    BKO_CHECK(nx >= 1 && ny >= 1 && nz >= 1 && m >= 1, "bad sizes");
    BKO_CHECK(static_cast<int64_t>(ldf) >= static_cast<int64_t>(nx) * ny * nz, "ldf must be >= n");
    BKO_CHECK(ksig > 0.0f, "ksig must be positive");
    return lstart_pack(nx, ny, nz, F, ldf, m, k_cell, kmu, ksig, hval, scale, x, static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

bko_status bko_lstart_pack_target(int n, const double *T, int ldt, int m, const double *scale, double gain, float *t,
                                  void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(T && scale && t, "NULL argument");
    BKO_CHECK(n >= 1 && m >= 1 && ldt >= n && gain > 0.0, "bad sizes");
    return lstart_pack_target(n, T, ldt, m, scale, gain, t, static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

bko_status bko_lstart_unpack(int n, const float *y, int m, const double *scale, double gain, double *X0, int ldx,
                             void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(y && scale && X0, "NULL argument");
    BKO_CHECK(n >= 1 && m >= 1 && ldx >= n && gain > 0.0, "bad sizes");
    return lstart_unpack(n, y, m, scale, gain, X0, ldx, static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

bko_status bko_jacobi_smooth(bko_op A, int m, const double *B, int ldb, double *X, int ldx, double *work, int ldw,
                             int sweeps, double omega, void *stream)
{
    BKO_GUARD_BEGIN
    BKO_CHECK(A != nullptr, "operator handle is NULL");
    const Operator &op = *reinterpret_cast<const Operator *>(A);
    BKO_CHECK(m >= 1 && B && X && work, "bad arguments");
    BKO_CHECK(ldb >= op.n && ldx >= op.n && ldw >= op.n, "leading dimensions must be >= n");
    BKO_CHECK(sweeps >= 0 && sweeps <= 10000, "sweeps outside [0, 10000]");
    BKO_CHECK(omega > 0.0 && omega < 2.0, "omega must be in (0, 2)");
    return launch_jacobi(op, m, B, ldb, X, ldx, work, ldw, sweeps, omega, static_cast<hipStream_t>(stream));
    BKO_GUARD_END
}

bko_status bko_timing_enable(int enable)
{
    TimingState &t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    t.mask = static_cast<unsigned>(enable);
    return BKO_OK;
}

bko_status bko_timing_set_stride(int every)
{
    BKO_CHECK(every >= 1, "timing stride must be >= 1, got %d", every);
    TimingState &t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    t.stride = static_cast<unsigned>(every);
    for (unsigned &c : t.counter) c = 0;
    return BKO_OK;
}

bko_status bko_timing_query(int family, int *launches, double *total_ms)
{
    BKO_CHECK(family >= 0 && family < kNumFamilies, "unknown timing family %d", family);
    TimingState &t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    bko_status st = drain(t);
    if (st != BKO_OK) return st;
    if (launches) *launches = t.launches[family];
    if (total_ms) *total_ms = t.total_ms[family];
    return BKO_OK;
}

bko_status bko_timing_reset(void)
{
    TimingState &t = timing();
    std::lock_guard<std::mutex> g(t.mu);
    bko_status st = drain(t);
    for (int f = 0; f < kNumFamilies; ++f) {
        t.launches[f] = 0;
        t.total_ms[f] = 0.0;
    }
    return st;
}

}  // extern "C"
