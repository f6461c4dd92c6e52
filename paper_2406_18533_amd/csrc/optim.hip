// Loss and optimizer kernels.
//  - L1 loss (paper section 2.1 step 3) with its gradient, batch loss = mean
//    of per-view losses (section 4: batch gradient = sum_k g_k / b).
//  - Adam with the batch scaling rules of section 4 (eqs. "lambda", "beta").
// Both are streaming, HBM-bound kernels: every element is read once and
// written once, with 16-byte accesses where the layout allows.
#include "common.hpp"

namespace gs {

// scratch[0] = 1 - b1^t, scratch[1] = sqrt(1 - b2^t); 0 in scratch[0] marks a skipped step.
__global__ void adam_prepare_kernel(int64_t *step, double b1, double b2, double *scratch, const int32_t *skip)
{
    if (skip && *skip != 0) {
        scratch[0] = 0.0;
        return;
    }
    int64_t t = *step + 1;
    *step = t;
    scratch[0] = 1.0 - pow(b1, (double)t);
    scratch[1] = sqrt(1.0 - pow(b2, (double)t));
}

AdamConst make_adam_const(const gs_adam_hparams *h)
{
    AdamConst c;
    double sb = sqrt((double)h->batch_size);
    for (int j = 0; j < 6; j++) c.lr[j] = h->lr[j] * sb;
    c.b1 = pow(h->beta1, (double)h->batch_size);
    c.b2 = pow(h->beta2, (double)h->batch_size);
    c.eps = h->eps;
    c.zero_grad = h->zero_grad;
    return c;
}

hipError_t launch_adam_prepare(int64_t *step, const AdamConst &c, double *scratch, const int32_t *skip, hipStream_t s)
{
    hipLaunchKernelGGL(adam_prepare_kernel, dim3(1), dim3(1), 0, s, step, c.b1, c.b2, scratch, skip);
    return hipGetLastError();
}

template <typename T, bool VEC>
__global__ void __launch_bounds__(256) adam_kernel(T *__restrict__ P, T *__restrict__ Gr, T *__restrict__ M,
                                                   T *__restrict__ Vv, int64_t n, AdamConst c,
                                                   const double *__restrict__ scratch)
{
    int row = blockIdx.y;
    double bc1 = scratch[0];
    if (bc1 == 0.0) {  // skipped step: only clear the gradient
        if (c.zero_grad)
            for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
                Gr[(int64_t)row * n + j] = T(0);
        return;
    }
    T b1 = (T)c.b1, b2 = (T)c.b2, eps = (T)c.eps;
    T step = adam_step_size<T>(c.lr[row_group(row)], bc1);
    T bc2s = adam_inv_bc2s<T>(scratch[1]);
    int64_t off = (int64_t)row * n;
    if (VEC) {
        using V = typename Vec4<T>::type;
        int64_t n4 = n / 4;
        for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n4; j += (int64_t)gridDim.x * blockDim.x) {
            V *pp = reinterpret_cast<V *>(P + off) + j, *gg = reinterpret_cast<V *>(Gr + off) + j;
            V *mm = reinterpret_cast<V *>(M + off) + j, *vv = reinterpret_cast<V *>(Vv + off) + j;
            V p = *pp, g = *gg, m = *mm, v = *vv;
            adam_one(p.x, g.x, m.x, v.x, b1, b2, step, bc2s, eps);
            adam_one(p.y, g.y, m.y, v.y, b1, b2, step, bc2s, eps);
            adam_one(p.z, g.z, m.z, v.z, b1, b2, step, bc2s, eps);
            adam_one(p.w, g.w, m.w, v.w, b1, b2, step, bc2s, eps);
            *pp = p;
            *mm = m;
            *vv = v;
            if (c.zero_grad) *gg = V{T(0), T(0), T(0), T(0)};
        }
    } else {
        for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
            int64_t k = off + j;
            T p = P[k], g = Gr[k], m = M[k], v = Vv[k];
            adam_one(p, g, m, v, b1, b2, step, bc2s, eps);
            P[k] = p;
            M[k] = m;
            Vv[k] = v;
            if (c.zero_grad) Gr[k] = T(0);
        }
    }
}

template <typename T>
hipError_t launch_adam(void *p, void *g, void *m, void *v, int64_t n, const gs_adam_hparams *h, int64_t *step,
                       double *scratch, const int32_t *skip, hipStream_t s)
{
    AdamConst c = make_adam_const(h);
    hipError_t e = launch_adam_prepare(step, c, scratch, skip, s);
    if (n == 0 || e != hipSuccess) return e;
    bool vec = (n % 4 == 0) && ((uintptr_t)p % 32 == 0) && ((uintptr_t)g % 32 == 0) && ((uintptr_t)m % 32 == 0) &&
               ((uintptr_t)v % 32 == 0);
    int64_t per_row = vec ? n / 4 : n;
    unsigned gx = (unsigned)((per_row + 255) / 256);
    if (gx > 4096) gx = 4096;
    if (gx == 0) gx = 1;
    if (vec)
        hipLaunchKernelGGL((adam_kernel<T, true>), dim3(gx, GS_PARAM_ROWS), dim3(256), 0, s, (T *)p, (T *)g, (T *)m,
                           (T *)v, n, c, (const double *)scratch);
    else
        hipLaunchKernelGGL((adam_kernel<T, false>), dim3(gx, GS_PARAM_ROWS), dim3(256), 0, s, (T *)p, (T *)g, (T *)m,
                           (T *)v, n, c, (const double *)scratch);
    return hipGetLastError();
}

// ------------------------------------------------------------------ L1 loss
constexpr int LOSS_BLOCKS = 64;

template <typename T>
__global__ void __launch_bounds__(256) l1_kernel(const T *__restrict__ rgb, const T *__restrict__ tgt,
                                                 T *__restrict__ dL, ViewTable vt, double scale,
                                                 double *__restrict__ partial)
{
    __shared__ double s_w[4];
    int v = blockIdx.y;
    int64_t beg = 3 * vt.pix_base[v], end = 3 * vt.pix_base[v + 1];
    int64_t cnt = end - beg;
    double wd = scale / ((double)cnt * (double)vt.nviews);
    T w = (T)wd;
    double acc = 0.0;
    for (int64_t j = beg + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < end;
         j += (int64_t)gridDim.x * blockDim.x) {
        T d = rgb[j] - tgt[j];
        dL[j] = d > T(0) ? w : (d < T(0) ? -w : T(0));
        acc += (double)(d < T(0) ? -d : d);
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0)
        partial[(int64_t)v * gridDim.x + blockIdx.x] = (s_w[0] + s_w[1] + s_w[2] + s_w[3]) * wd;
}

__global__ void l1_finish_kernel(const double *partial, int64_t n, double *loss)
{
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int64_t j = 0; j < n; j++) s += partial[j];
    *loss = s;
}

size_t loss_ws_bytes(int32_t views) { return sizeof(double) * (size_t)LOSS_BLOCKS * (size_t)views; }

template <typename T>
hipError_t launch_l1(const void *rgb, const void *tgt, const ViewTable &vt, double scale, void *dL, double *loss,
                     void *ws, hipStream_t s)
{
    hipLaunchKernelGGL(l1_kernel<T>, dim3(LOSS_BLOCKS, vt.nviews), dim3(256), 0, s, (const T *)rgb, (const T *)tgt,
                       (T *)dL, vt, scale, (double *)ws);
    hipLaunchKernelGGL(l1_finish_kernel, dim3(1), dim3(64), 0, s, (const double *)ws,
                       (int64_t)LOSS_BLOCKS * vt.nviews, loss);
    return hipGetLastError();
}

template hipError_t launch_adam<float>(void *, void *, void *, void *, int64_t, const gs_adam_hparams *, int64_t *,
                                       double *, const int32_t *, hipStream_t);
template hipError_t launch_adam<double>(void *, void *, void *, void *, int64_t, const gs_adam_hparams *, int64_t *,
                                        double *, const int32_t *, hipStream_t);
template hipError_t launch_l1<float>(const void *, const void *, const ViewTable &, double, void *, double *, void *,
                                     hipStream_t);
template hipError_t launch_l1<double>(const void *, const void *, const ViewTable &, double, void *, double *, void *,
                                      hipStream_t);

}  // namespace gs
