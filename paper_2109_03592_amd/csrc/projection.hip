// projection.hip -- projection onto previous solutions (section 2 of the
// paper accelerates successive solves this way, after Fischer).
//
// A basis x_1..x_l of earlier solutions is kept A-orthonormal together with
// A x_i.  For a new right-hand side the guess xbar = sum_i (x_i . b) x_i is
// the element of the span closest to the solution in the A-norm; PCG then
// starts from it.  A solution joins the basis after two passes of
// Gram-Schmidt in the A-inner product (x_i^T A v = x_i . (A v), unique-dof
// inner products) and A-normalisation; a remainder whose A-norm fell below
// drop_tol times the vector's own is dropped; a full basis restarts.
//
// Kernels: one pass computes all l inner products against a vector (each
// workgroup writes l partials, l single-workgroup sums in a fixed order);
// one pass forms a combination of the basis, or removes it from v and A v.
#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels.hpp"
#include "operator.hpp"
#include "sem_internal.hpp"

namespace sem {

constexpr int kMaxProj = 32;

struct ProjPtrs {
    const double *v[kMaxProj];
};

__device__ inline double inv_mult_p(uint8_t m) { return 1.0 / (double)m; }

// partial[b * l + i] = sum over this workgroup's points of V_i y / mult
__global__ __launch_bounds__(256) void multi_dot_kernel(int64_t n, int l, ProjPtrs V, const double *__restrict__ y,
                                                        const uint8_t *__restrict__ mult,
                                                        double *__restrict__ partial)
{
    double acc[kMaxProj];
#pragma unroll
    for (int i = 0; i < kMaxProj; ++i) acc[i] = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        const double yq = y[q] * inv_mult_p(mult[q]);
#pragma unroll
        for (int i = 0; i < kMaxProj; ++i)
            if (i < l) acc[i] += V.v[i][q] * yq;
    }
#pragma unroll
    for (int i = 0; i < kMaxProj; ++i)
        if (i < l) {  // uniform over the workgroup
            double v[1] = {acc[i]};
            block_reduce_store<1>(v, partial + i, l);
            __syncthreads();
        }
}

// out[i] = sum over workgroups of partial[b * l + i] (workgroup i, fixed order)
__global__ __launch_bounds__(256) void multi_reduce_kernel(const double *__restrict__ partial, int64_t blocks, int l,
                                                           double *__restrict__ out)
{
    __shared__ double red[256];
    const int i = blockIdx.x;
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < blocks; b += blockDim.x) s += partial[b * l + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = red[0];
}

// out = sum_i c_i V_i
__global__ __launch_bounds__(256) void combine_kernel(int64_t n, int l, ProjPtrs V, const double *__restrict__ c,
                                                      double *__restrict__ out)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < kMaxProj; ++i)
            if (i < l) s += c[i] * V.v[i][q];
        out[q] = s;
    }
}

// v -= sum_i c_i X_i, Av -= sum_i c_i AX_i
__global__ __launch_bounds__(256) void remove_kernel(int64_t n, int l, ProjPtrs X, ProjPtrs AX,
                                                     const double *__restrict__ c, double *__restrict__ v,
                                                     double *__restrict__ Av)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        double a = v[q], b = Av[q];
#pragma unroll
        for (int i = 0; i < kMaxProj; ++i)
            if (i < l) {
                a -= c[i] * X.v[i][q];
                b -= c[i] * AX.v[i][q];
            }
        v[q] = a;
        Av[q] = b;
    }
}

__global__ void scale2_kernel(int64_t n, double s, double *__restrict__ a, double *__restrict__ b)
{
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (int64_t)gridDim.x * blockDim.x) {
        a[q] *= s;
        b[q] *= s;
    }
}

template <typename F>
static sem_status pguard(F &&f)
{
    try {
        return f();
    } catch (const Failure &x) {
        return x.status;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return SEM_ENOMEM;
    } catch (const std::exception &x) {
        set_error(x.what());
        return SEM_EINVAL;
    } catch (...) {
        set_error("unknown internal error");
        return SEM_EINVAL;
    }
}

}  // namespace sem

struct sem_proj {
    sem_mesh *mesh = nullptr;
    int max_vectors = 0;
    int l = 0;                  // basis vectors held
    int op_version = 0;         // operator the basis was built for
    double drop_tol = 1e-8;
    std::vector<double *> X, AX;
    double *coef = nullptr;     // [kMaxProj]
    double *partial = nullptr;  // [blocks * kMaxProj]
    double *scal = nullptr;     // [2]
    int64_t blocks = 0;
};

namespace sem {

static ProjPtrs ptrs(const std::vector<double *> &v, int l)
{
    ProjPtrs p{};
    for (int i = 0; i < l; ++i) p.v[i] = v[i];
    return p;
}

static void sync_version(sem_proj *P)
{
    if (P->op_version != P->mesh->op_version) {
        P->l = 0;
        P->op_version = P->mesh->op_version;
    }
}

// coef[0..l) = X_i . y
static void multi_dot(sem_proj *P, int l, const double *y, hipStream_t s)
{
    const int64_t n = P->mesh->h.nL;
    hipLaunchKernelGGL(multi_dot_kernel, dim3((unsigned)P->blocks), dim3(256), 0, s, n, l, ptrs(P->X, l), y,
                       P->mesh->mult, P->partial);
    SEM_HIP(hipGetLastError());
    hipLaunchKernelGGL(multi_reduce_kernel, dim3(l), dim3(256), 0, s, P->partial, P->blocks, l, P->coef);
    SEM_HIP(hipGetLastError());
}

static double dot_host(sem_proj *P, const double *a, const double *b, hipStream_t s)
{
    SEM_HIP(launch_dot_unique<double>(P->mesh->h.nL, a, b, P->mesh->mult, P->partial, P->scal, s));
    double v = 0.0;
    SEM_HIP(hipMemcpyAsync(&v, P->scal, sizeof(double), hipMemcpyDeviceToHost, s));
    SEM_HIP(hipStreamSynchronize(s));
    return v;
}

static void project(sem_proj *P, const double *b, double *x, hipStream_t s)
{
    const int64_t n = P->mesh->h.nL;
    if (P->l == 0) {
        SEM_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
        return;
    }
    multi_dot(P, P->l, b, s);
    hipLaunchKernelGGL(combine_kernel, dim3(vec_blocks(n)), dim3(256), 0, s, n, P->l, ptrs(P->X, P->l), P->coef, x);
    SEM_HIP(hipGetLastError());
}

// returns 1 when x joined the basis, 0 when it was dropped
static int add(sem_proj *P, const double *x, hipStream_t s)
{
    sem_mesh *m = P->mesh;
    const int64_t n = m->h.nL;
    if (P->l >= P->max_vectors) P->l = 0;
    const int l = P->l;
    double *v = P->X[l], *Av = P->AX[l];
    SEM_HIP(hipMemcpyAsync(v, x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    const sem_status st = sem_axgs(m, SEM_FP64, v, Av, s);
    if (st != SEM_OK) fail(st, "sem_proj_add: operator apply failed");
    const double n0 = dot_host(P, v, Av, s);
    if (!(n0 > 0.0) || !std::isfinite(n0)) return 0;
    if (l > 0) {
        for (int pass = 0; pass < 2; ++pass) {
            multi_dot(P, l, Av, s);
            hipLaunchKernelGGL(remove_kernel, dim3(vec_blocks(n)), dim3(256), 0, s, n, l, ptrs(P->X, l),
                               ptrs(P->AX, l), P->coef, v, Av);
            SEM_HIP(hipGetLastError());
        }
    }
    const double n2 = dot_host(P, v, Av, s);
    if (!(n2 > P->drop_tol * P->drop_tol * n0)) return 0;
    hipLaunchKernelGGL(scale2_kernel, dim3(vec_blocks(n)), dim3(256), 0, s, n, 1.0 / std::sqrt(n2), v, Av);
    SEM_HIP(hipGetLastError());
    SEM_HIP(hipStreamSynchronize(s));
    P->l = l + 1;
    return 1;
}

}  // namespace sem

using namespace sem;

extern "C" {

sem_status sem_proj_create(sem_mesh *mesh, int max_vectors, sem_proj **out)
{
    return pguard([&]() -> sem_status {
        if (!mesh || !out) fail(SEM_EINVAL, "sem_proj_create: null argument");
        if (max_vectors < 1 || max_vectors > kMaxProj) fail(SEM_EINVAL, "sem_proj_create: max_vectors must be 1..32");
        *out = nullptr;
        sem_proj *P = new sem_proj();
        P->mesh = mesh;
        P->max_vectors = max_vectors;
        P->op_version = mesh->op_version;
        const int64_t n = mesh->h.nL;
        P->blocks = vec_blocks(n);
        auto alloc = [&](size_t bytes) {
            void *p = nullptr;
            if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) {
                (void)hipGetLastError();
                return (double *)nullptr;
            }
            return (double *)p;
        };
        bool ok = true;
        for (int i = 0; i < max_vectors && ok; ++i) {
            double *a = alloc(sizeof(double) * n), *b = alloc(sizeof(double) * n);
            if (a) P->X.push_back(a);
            if (b) P->AX.push_back(b);
            ok = a && b;
        }
        if (ok) ok = (P->coef = alloc(sizeof(double) * kMaxProj)) != nullptr;
        if (ok) ok = (P->partial = alloc(sizeof(double) * (size_t)P->blocks * kMaxProj)) != nullptr;
        if (ok) ok = (P->scal = alloc(sizeof(double) * 2)) != nullptr;
        if (!ok) {
            sem_proj_free(P);
            fail(SEM_ENOMEM, "sem_proj_create: device allocation failed");
        }
        *out = P;
        return SEM_OK;
    });
}

sem_status sem_proj_free(sem_proj *P)
{
    if (!P) return SEM_OK;
    for (double *p : P->X) hipFree(p);
    for (double *p : P->AX) hipFree(p);
    if (P->coef) hipFree(P->coef);
    if (P->partial) hipFree(P->partial);
    if (P->scal) hipFree(P->scal);
    delete P;
    return SEM_OK;
}

sem_status sem_proj_reset(sem_proj *P)
{
    return pguard([&]() -> sem_status {
        if (!P) fail(SEM_EINVAL, "sem_proj_reset: null handle");
        P->l = 0;
        return SEM_OK;
    });
}

sem_status sem_proj_size(sem_proj *P, int *n)
{
    return pguard([&]() -> sem_status {
        if (!P || !n) fail(SEM_EINVAL, "sem_proj_size: null argument");
        sync_version(P);
        *n = P->l;
        return SEM_OK;
    });
}

sem_status sem_proj_project(sem_proj *P, const double *b, double *x, void *stream)
{
    return pguard([&]() -> sem_status {
        if (!P || !b || !x) fail(SEM_EINVAL, "sem_proj_project: null argument");
        sync_version(P);
        project(P, b, x, (hipStream_t)stream);
        return SEM_OK;
    });
}

sem_status sem_proj_add(sem_proj *P, const double *x, int *added, void *stream)
{
    return pguard([&]() -> sem_status {
        if (!P || !x) fail(SEM_EINVAL, "sem_proj_add: null argument");
        sync_version(P);
        const int a = add(P, x, (hipStream_t)stream);
        if (added) *added = a;
        return SEM_OK;
    });
}

sem_status sem_proj_solve(sem_proj *P, const double *b, double *x, const sem_solve_opts *opts, sem_solve_stats *stats,
                          void *stream)
{
    return pguard([&]() -> sem_status {
        if (!P || !b || !x) fail(SEM_EINVAL, "sem_proj_solve: null argument");
        hipStream_t s = (hipStream_t)stream;
        sync_version(P);
        sem_solve_opts o;
        sem_solve_opts_default(&o);
        if (opts) o = *opts;
        o.x0_given = 1;
        project(P, b, x, s);
        const sem_status st = sem_pcg_solve(P->mesh, b, x, &o, stats, stream);
        if (st == SEM_OK) add(P, x, s);
        return st;
    });
}

}  // extern "C"
