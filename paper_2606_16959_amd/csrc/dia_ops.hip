// Kernels on general operators in the diagonal layout (complex, FP64 or
// FP32): construction from Pauli terms, SpGEMM, sum, scaling, largest-entry
// norm and precision conversion.  Used by the truncated-Taylor exponential
// (paper: Alg. 2) and the single-propagator simulation loop (Alg. 3).
#include <hip/hip_runtime.h>

#include "hs_internal.h"

namespace hs {

namespace {

struct Z {
    double re, im;
};

__device__ __forceinline__ Z zmul(Z a, Z b) { return Z{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

}  // namespace

// H[r, r+d] = sum over terms with X-mask (r xor (r+d)) of c i^ny (-1)^{popcount((r+d) & z)}.
// Terms are sorted by X-mask; cls_mask[j] is the j-th distinct mask and its
// terms are [cls_ptr[j], cls_ptr[j+1]).
__global__ void pauli_dia_kernel(PauliDiaArgs a) {
    const int j = blockIdx.y;
    const int64_t d = a.offs[j];
    const int64_t len = a.N - (d < 0 ? -d : d);
    const int64_t neg = d < 0 ? d : 0;
    double *out = a.out[j];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i - neg, p = r + d;
        const uint64_t m = (uint64_t)(r ^ p);
        double vr = 0.0, vi = 0.0;
        for (int c = 0; c < a.n_cls; ++c) {
            if (a.cls_mask[c] != m) continue;
            for (int k = a.cls_ptr[c]; k < a.cls_ptr[c + 1]; ++k) {
                const double s = (__popcll((uint64_t)p & a.zmask[k]) & 1) ? -a.coeff[k] : a.coeff[k];
                switch (a.ny[k] & 3) {          // times i^ny
                    case 0: vr += s; break;
                    case 1: vi += s; break;
                    case 2: vr -= s; break;
                    default: vi -= s; break;
                }
            }
            break;
        }
        out[2 * i] = vr;
        out[2 * i + 1] = vi;
    }
}

// C[r, r+c] = scale * sum_{(a,b): a+b=c} A[r, r+a] B[r+a, r+c]; one result
// diagonal per blockIdx.y; contributors of result j are [cptr[j], cptr[j+1]).
// With store == false only the largest entry modulus per block is written.
__global__ void spgemm_kernel(SpgemmArgs a, bool store) {
    const int j = blockIdx.y;
    const int64_t c = a.c_offs[j];
    const int64_t N = a.N;
    const int64_t len = N - (c < 0 ? -c : c);
    const int64_t negc = c < 0 ? c : 0;
    double *out = store ? a.c_ptr[j] : nullptr;
    double vmax = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = i - negc;
        Z acc{0.0, 0.0};
        for (int q = a.cptr[j]; q < a.cptr[j + 1]; ++q) {
            const int ia = a.pairs[2 * q], ib = a.pairs[2 * q + 1];
            const int64_t da = a.a_offs[ia];
            const int64_t ra = r + da;                    // column of A = row of B
            if (ra < 0 || ra >= N) continue;
            const int64_t ea = r < ra ? r : ra;           // storage index min(row, col)
            const int64_t eb = ra < r + c ? ra : r + c;
            const double *pa = a.a_ptr[ia] + 2 * ea;
            const double *pb = a.b_ptr[ib] + 2 * eb;
            acc = Z{acc.re + (pa[0] * pb[0] - pa[1] * pb[1]), acc.im + (pa[0] * pb[1] + pa[1] * pb[0])};
        }
        acc = zmul(acc, Z{a.scale_re, a.scale_im});
        if (store) {
            out[2 * i] = acc.re;
            out[2 * i + 1] = acc.im;
        }
        vmax = fmax(vmax, sqrt(acc.re * acc.re + acc.im * acc.im));
    }
    __shared__ double red[256];
    red[threadIdx.x] = vmax;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) a.block_max[(int64_t)j * gridDim.x + blockIdx.x] = red[0];
}

// out_j = (ia[j] >= 0 ? A[ia[j]] : 0) + (ib[j] >= 0 ? B[ib[j]] : 0), diagonal by diagonal.
__global__ void dia_add_kernel(DiaAddArgs a) {
    const int j = blockIdx.y;
    const int64_t d = a.offs[j];
    const int64_t len = a.N - (d < 0 ? -d : d);
    const double *pa = a.ia[j] >= 0 ? a.a_ptr[a.ia[j]] : nullptr;
    const double *pb = a.ib[j] >= 0 ? a.b_ptr[a.ib[j]] : nullptr;
    double *out = a.out[j];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 2 * len;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (pa ? pa[i] : 0.0) + (pb ? pb[i] : 0.0);
}

// largest entry modulus of every stored entry: per-block maxima
__global__ void dia_maxabs_kernel(const double *const *ptrs, const int64_t *offs, int64_t N,
                                  double *block_max) {
    const int j = blockIdx.y;
    const int64_t d = offs[j];
    const int64_t len = N - (d < 0 ? -d : d);
    const double *p = ptrs[j];
    double vmax = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x)
        vmax = fmax(vmax, sqrt(p[2 * i] * p[2 * i] + p[2 * i + 1] * p[2 * i + 1]));
    __shared__ double red[256];
    red[threadIdx.x] = vmax;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) block_max[(int64_t)j * gridDim.x + blockIdx.x] = red[0];
}

// FP64 diagonals -> FP32 diagonals (round to nearest)
__global__ void dia_to_c64_kernel(const double *const *src, float *const *dst, const int64_t *offs,
                                  int64_t N) {
    const int j = blockIdx.y;
    const int64_t d = offs[j];
    const int64_t len = 2 * (N - (d < 0 ? -d : d));
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[j][i] = (float)src[j][i];
}

__global__ void dia_fill_kernel(double *out, int64_t len, double re, double im) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x) {
        out[2 * i] = re;
        out[2 * i + 1] = im;
    }
}

// exact exponential of a diagonal operator: out = exp(-i dt h), elementwise
__global__ void diag_exp_kernel(const double *h, double *out, int64_t len, double dt) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x) {
        // -i dt (a + ib) = dt b - i dt a
        const double mag = exp(dt * h[2 * i + 1]);
        double s, c;
        sincos(-dt * h[2 * i], &s, &c);
        out[2 * i] = mag * c;
        out[2 * i + 1] = mag * s;
    }
}

static inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

int launch_dia_fill(double *out, int64_t len, double re, double im, void *stream) {
    hipLaunchKernelGGL(dia_fill_kernel, dim3(dia_grid_x(len)), dim3(256), 0, S(stream), out, len, re, im);
    return (int)hipGetLastError();
}

int launch_diag_exp(const double *h, double *out, int64_t len, double dt, void *stream) {
    hipLaunchKernelGGL(diag_exp_kernel, dim3(dia_grid_x(len)), dim3(256), 0, S(stream), h, out, len, dt);
    return (int)hipGetLastError();
}

int dia_grid_x(int64_t len) {
    int64_t g = (len + 255) / 256;
    if (g < 1) g = 1;
    if (g > 1024) g = 1024;
    return (int)g;
}

int launch_pauli_dia(const PauliDiaArgs &a, int nd, void *stream) {
    hipLaunchKernelGGL(pauli_dia_kernel, dim3(dia_grid_x(a.N), nd), dim3(256), 0, S(stream), a);
    return (int)hipGetLastError();
}

int launch_spgemm(const SpgemmArgs &a, int nd, int gx, bool store, void *stream) {
    hipLaunchKernelGGL(spgemm_kernel, dim3(gx, nd), dim3(256), 0, S(stream), a, store);
    return (int)hipGetLastError();
}

int launch_dia_add(const DiaAddArgs &a, int nd, void *stream) {
    hipLaunchKernelGGL(dia_add_kernel, dim3(dia_grid_x(2 * a.N), nd), dim3(256), 0, S(stream), a);
    return (int)hipGetLastError();
}

int launch_dia_maxabs(const double *const *ptrs, const int64_t *offs, int64_t N, int nd, int gx,
                      double *block_max, void *stream) {
    hipLaunchKernelGGL(dia_maxabs_kernel, dim3(gx, nd), dim3(256), 0, S(stream), ptrs, offs, N, block_max);
    return (int)hipGetLastError();
}

int launch_dia_to_c64(const double *const *src, float *const *dst, const int64_t *offs, int64_t N,
                      int nd, void *stream) {
    hipLaunchKernelGGL(dia_to_c64_kernel, dim3(dia_grid_x(2 * N), nd), dim3(256), 0, S(stream), src, dst,
                       offs, N);
    return (int)hipGetLastError();
}

}  // namespace hs
