// net.hip -- learned PCG warm start: a bias-free 6-layer 3x3 convolutional net over the
// control-point grid (3 -> 32 -> 32 -> 32 -> 32 -> 32 -> 3 channels, zero padding, LeakyReLU
// with slope 0.1 between layers), FP32 forward, backward (data and weights), loss and Adam.
// This is a method extension (the paper has no learned component).
//
// Layouts: activations [b][channel][j][i] (a CP grid of n_v rows and n_u columns per channel),
// weights per layer [c_out][c_in][3][3], layers concatenated.
// Forward conv: one 16 x 16 pixel tile per workgroup; the input tile plus a one-pixel halo is
// staged in LDS for all input channels, every thread owns one pixel and all output channels,
// and the weights (uniform across the workgroup) are read through the scalar cache.
// Weight gradient: per-tile partial sums written to scratch, then reduced over tiles in a
// fixed order (deterministic, no atomics).
// The input is normalised per sample by its RMS; since the net is bias-free with LeakyReLU it is
// positively homogeneous, so the normalisation only keeps FP32 in range.
#include "bsc_internal.h"

#include <mutex>
#include <string>

namespace bsc {
namespace {

constexpr int kT = 16;                // output tile edge
constexpr int kHalo = kT + 2;
constexpr int kPlane = kHalo * kHalo + 1;   // padded LDS plane (odd stride against bank conflicts)
constexpr int kC = 32;                // hidden channels
constexpr float kSlope = 0.1f;
constexpr int kLayers = 6;
constexpr int kCin[kLayers] = {3, 32, 32, 32, 32, 32};
constexpr int kCout[kLayers] = {32, 32, 32, 32, 32, 3};

__host__ __device__ constexpr int layer_offset(int l) {
    int o = 0;
    for (int k = 0; k < l; ++k) o += kCin[k] * kCout[k] * 9;
    return o;
}

// Per-sample 1/RMS of the input (3 n_cp values per sample); scale[b].
__global__ void __launch_bounds__(256) k_rms(const float *__restrict__ in, int n, float *__restrict__ scale) {
    __shared__ double sh[4];
    const float *p = in + size_t(blockIdx.x) * 3 * n;
    double v = 0.0;
    for (int t = threadIdx.x; t < 3 * n; t += blockDim.x) v += double(p[t]) * double(p[t]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double tot = sh[0] + sh[1] + sh[2] + sh[3];
        const double rms = sqrt(tot / (3.0 * n));
        scale[blockIdx.x] = rms > 0.0 ? float(1.0 / rms) : 0.0f;
    }
}

// Loads a (kHalo x kHalo) input tile with zero padding for CIN channels into LDS.
template <int CIN>
__device__ __forceinline__ void load_tile(const float *__restrict__ src, int n_u, int n_v, int i0, int j0, float s,
                                          float *lds) {
    const size_t plane = size_t(n_u) * n_v;
    for (int t = threadIdx.x; t < CIN * kHalo * kHalo; t += blockDim.x) {
        const int c = t / (kHalo * kHalo), rem = t % (kHalo * kHalo);
        const int ly = rem / kHalo, lx = rem % kHalo;
        const int gi = i0 + lx - 1, gj = j0 + ly - 1;
        float v = 0.0f;
        if (gi >= 0 && gi < n_u && gj >= 0 && gj < n_v) v = src[c * plane + size_t(gj) * n_u + gi] * s;
        lds[c * kPlane + ly * kHalo + lx] = v;
    }
}

// 3x3 convolution, zero padding. EPI: 0 plain, 1 LeakyReLU, 2 multiply by the LeakyReLU slope
// of aux (aux = the activation whose pre-activation gradient is wanted). Weights in the
// reordered layout wr[ci][tap][co], so the COUT weights of one (ci, tap) are contiguous.
// in_scale (nullable): per-sample factor applied to the input (RMS normalisation).
template <int CIN, int COUT, int EPI>
__global__ void __launch_bounds__(kT *kT) k_conv(int n_u, int n_v, const float *__restrict__ in, const float *__restrict__ w,
                                                 float *__restrict__ out, const float *__restrict__ aux,
                                                 const float *__restrict__ in_scale) {
    __shared__ float lds[CIN * kPlane];
    const int b = blockIdx.z;
    const size_t plane = size_t(n_u) * n_v;
    const int i0 = blockIdx.x * kT, j0 = blockIdx.y * kT;
    const float s = in_scale ? in_scale[b] : 1.0f;
    load_tile<CIN>(in + size_t(b) * CIN * plane, n_u, n_v, i0, j0, s, lds);
    __syncthreads();
    const int tx = threadIdx.x % kT, ty = threadIdx.x / kT;
    float acc[COUT];
#pragma unroll
    for (int co = 0; co < COUT; ++co) acc[co] = 0.0f;
    for (int ci = 0; ci < CIN; ++ci) {
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const float v = lds[ci * kPlane + (ty + tap / 3) * kHalo + (tx + tap % 3)];
#pragma unroll
            for (int co = 0; co < COUT; ++co) acc[co] += w[(ci * 9 + tap) * COUT + co] * v;
        }
    }
    const int gi = i0 + tx, gj = j0 + ty;
    if (gi >= n_u || gj >= n_v) return;
    const size_t pix = size_t(gj) * n_u + gi;
    float *o = out + size_t(b) * COUT * plane;
#pragma unroll
    for (int co = 0; co < COUT; ++co) {
        float v = acc[co];
        if (EPI == 1) v = v > 0.0f ? v : kSlope * v;
        if (EPI == 2) v = aux[size_t(b) * COUT * plane + co * plane + pix] > 0.0f ? v : kSlope * v;
        o[co * plane + pix] = v;
    }
}

// Weight reorder for k_conv. flip = 0: forward, wr[ci][tap][co] = w[co][ci][tap].
// flip = 1: backward data of the layer (a conv from cout to cin channels with flipped taps),
// wr[co][8 - tap][ci] = w[co][ci][tap].
__global__ void k_reorder(const float *__restrict__ w, float *__restrict__ wr, int cin, int cout, int flip) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cin * cout * 9) return;
    const int tap = t % 9, ci = (t / 9) % cin, co = t / (9 * cin);
    if (flip) wr[(co * 9 + (8 - tap)) * cin + ci] = w[t];
    else wr[(ci * 9 + tap) * cout + co] = w[t];
}

void reorder_all(const float *w, float *wr, int flip, hipStream_t st) {
    for (int l = 0; l < kLayers; ++l) {
        const int len = kCin[l] * kCout[l] * 9;
        k_reorder<<<(len + 255) / 256, 256, 0, st>>>(w + layer_offset(l), wr + layer_offset(l), kCin[l], kCout[l], flip);
    }
}

// Per-tile partial weight gradient dW[co][ci][tap] = sum_p dZ[co][p] X[ci][p + off(tap)],
// X optionally scaled per sample. part[(b * tiles + tile) * COUT*CIN*9 + k].
template <int CIN, int COUT>
__global__ void __launch_bounds__(kT *kT) k_dw_tile(int n_u, int n_v, const float *__restrict__ X, const float *__restrict__ dZ,
                                                    const float *__restrict__ x_scale, float *__restrict__ part) {
    __shared__ float lx[CIN * kPlane];
    __shared__ float lz[COUT * kT * kT];
    const int b = blockIdx.z;
    const size_t plane = size_t(n_u) * n_v;
    const int i0 = blockIdx.x * kT, j0 = blockIdx.y * kT;
    const float s = x_scale ? x_scale[b] : 1.0f;
    load_tile<CIN>(X + size_t(b) * CIN * plane, n_u, n_v, i0, j0, s, lx);
    for (int t = threadIdx.x; t < COUT * kT * kT; t += blockDim.x) {
        const int c = t / (kT * kT), rem = t % (kT * kT);
        const int gi = i0 + rem % kT, gj = j0 + rem / kT;
        lz[t] = (gi < n_u && gj < n_v) ? dZ[size_t(b) * COUT * plane + c * plane + size_t(gj) * n_u + gi] : 0.0f;
    }
    __syncthreads();
    const int tiles = gridDim.x * gridDim.y, tile = blockIdx.y * gridDim.x + blockIdx.x;
    float *dst = part + (size_t(b) * tiles + tile) * (COUT * CIN * 9);
    // each thread: one input channel ci and a group of up to 4 output channels, 9 taps each
    constexpr int kGroupsCo = (COUT + 3) / 4;
    for (int job = threadIdx.x; job < CIN * kGroupsCo; job += blockDim.x) {
        const int ci = job % CIN, cg = job / CIN;
        float acc[4][9];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) acc[q][tap] = 0.0f;
        for (int py = 0; py < kT; ++py) {
            for (int px = 0; px < kT; ++px) {
                float xv[9];
#pragma unroll
                for (int tap = 0; tap < 9; ++tap) xv[tap] = lx[ci * kPlane + (py + tap / 3) * kHalo + (px + tap % 3)];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int co = 4 * cg + q;
                    if (co < COUT) {
                        const float z = lz[co * kT * kT + py * kT + px];
#pragma unroll
                        for (int tap = 0; tap < 9; ++tap) acc[q][tap] += z * xv[tap];
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int co = 4 * cg + q;
            if (co < COUT) {
#pragma unroll
                for (int tap = 0; tap < 9; ++tap) dst[(co * CIN + ci) * 9 + tap] = acc[q][tap];
            }
        }
    }
}

// dw[k] = sum over n partial rows (fixed order).
__global__ void k_dw_reduce(const float *__restrict__ part, int n, int len, float *__restrict__ dw) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= len) return;
    double s = 0.0;
    for (int t = 0; t < n; ++t) s += part[size_t(t) * len + k];
    dw[k] = float(s);
}

// Loss of the best scalar multiple: per sample, with pinned CPs (input exactly zero) masked,
// L = 1 - (p.t)^2 / (|p|^2 |t|^2); stage 1 writes per-block partials of p.t, p.p, t.t.
__global__ void __launch_bounds__(256) k_loss_part(int n, const float *__restrict__ pred, const float *__restrict__ tgt,
                                                   const float *__restrict__ in, double *__restrict__ part, int nb) {
    __shared__ double sh[3][4];
    const int b = blockIdx.y;
    const float *P = pred + size_t(b) * 3 * n, *Tg = tgt + size_t(b) * 3 * n, *I = in + size_t(b) * 3 * n;
    double v[3] = {0.0, 0.0, 0.0};
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < n; a += gridDim.x * blockDim.x) {
        const bool free_cp = I[a] != 0.0f || I[n + a] != 0.0f || I[2 * n + a] != 0.0f;
        if (!free_cp) continue;
        for (int c = 0; c < 3; ++c) {
            const double p = P[c * n + a], t = Tg[c * n + a];
            v[0] += p * t; v[1] += p * p; v[2] += t * t;
        }
    }
    for (int k = 0; k < 3; ++k) {
        double x = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off);
        if ((threadIdx.x & 63) == 0) sh[k][threadIdx.x >> 6] = x;
    }
    __syncthreads();
    if (threadIdx.x < 3)
        part[(size_t(b) * nb + blockIdx.x) * 3 + threadIdx.x] = sh[threadIdx.x][0] + sh[threadIdx.x][1] + sh[threadIdx.x][2] + sh[threadIdx.x][3];
}

// Stage 2: per-sample sums, mean loss and dL/dpred (zero on masked CPs).
__global__ void __launch_bounds__(256) k_loss_grad(int n, int batch, const float *__restrict__ pred, const float *__restrict__ tgt,
                                                   const float *__restrict__ in, const double *__restrict__ part, int nb,
                                                   float *__restrict__ loss, float *__restrict__ dpred) {
    const int b = blockIdx.y;
    double pt = 0.0, pp = 0.0, tt = 0.0;
    for (int k = 0; k < nb; ++k) {
        pt += part[(size_t(b) * nb + k) * 3];
        pp += part[(size_t(b) * nb + k) * 3 + 1];
        tt += part[(size_t(b) * nb + k) * 3 + 2];
    }
    const double den = pp * tt;
    const double c1 = den > 0.0 ? -2.0 * pt / den : 0.0;            // coefficient of t
    const double c2 = den > 0.0 ? 2.0 * pt * pt / (pp * den) : 0.0;   // coefficient of p
    if (blockIdx.x == 0 && threadIdx.x == 0 && b == 0) {
        double L = 0.0;
        for (int bb = 0; bb < batch; ++bb) {
            double a = 0.0, q = 0.0, r = 0.0;
            for (int k = 0; k < nb; ++k) {
                a += part[(size_t(bb) * nb + k) * 3];
                q += part[(size_t(bb) * nb + k) * 3 + 1];
                r += part[(size_t(bb) * nb + k) * 3 + 2];
            }
            L += (q * r > 0.0) ? 1.0 - a * a / (q * r) : 1.0;
        }
        loss[0] = float(L / batch);
    }
    const float *P = pred + size_t(b) * 3 * n, *Tg = tgt + size_t(b) * 3 * n, *I = in + size_t(b) * 3 * n;
    float *D = dpred + size_t(b) * 3 * n;
    for (int a = blockIdx.x * blockDim.x + threadIdx.x; a < n; a += gridDim.x * blockDim.x) {
        const bool free_cp = I[a] != 0.0f || I[n + a] != 0.0f || I[2 * n + a] != 0.0f;
        for (int c = 0; c < 3; ++c)
            D[c * n + a] = free_cp ? float((c1 * Tg[c * n + a] + c2 * P[c * n + a]) / batch) : 0.0f;
    }
}

__global__ void k_adam(int n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gt = g[t];
    const float mt = b1 * m[t] + (1.0f - b1) * gt;
    const float vt = b2 * v[t] + (1.0f - b2) * gt * gt;
    m[t] = mt;
    v[t] = vt;
    p[t] -= lr * (mt / c1) / (sqrtf(vt / c2) + eps);
}

inline dim3 conv_grid(int n_u, int n_v, int batch) { return dim3((n_u + kT - 1) / kT, (n_v + kT - 1) / kT, batch); }

template <int CIN, int COUT, int EPI>
void conv(int n_u, int n_v, int batch, const float *in, const float *w, float *out, const float *aux, const float *sc,
          hipStream_t st) {
    k_conv<CIN, COUT, EPI><<<conv_grid(n_u, n_v, batch), kT * kT, 0, st>>>(n_u, n_v, in, w, out, aux, sc);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct NetScratch {
    float *dz0, *dz1, *wt, *scale, *part;
    double *lpart;
};

NetScratch carve(void *base, int n_u, int n_v, int batch) {
    const size_t n = size_t(n_u) * n_v;
    const size_t tiles = size_t((n_u + kT - 1) / kT) * ((n_v + kT - 1) / kT);
    char *p = (char *)base;
    NetScratch s;
    s.dz0 = (float *)p; p += align256(4 * kC * n * batch);
    s.dz1 = (float *)p; p += align256(4 * kC * n * batch);
    s.wt = (float *)p; p += align256(4 * BSC_NET_PARAMS);
    s.scale = (float *)p; p += align256(4 * size_t(batch));
    s.part = (float *)p; p += align256(4 * tiles * batch * kC * kC * 9);
    s.lpart = (double *)p;
    return s;
}

}  // namespace

size_t net_scratch_bytes(int n_u, int n_v, int batch) {
    const size_t n = size_t(n_u) * n_v;
    const size_t tiles = size_t((n_u + kT - 1) / kT) * ((n_v + kT - 1) / kT);
    return 2 * align256(4 * kC * n * batch) + align256(4 * BSC_NET_PARAMS) + align256(4 * size_t(batch)) +
           align256(4 * tiles * batch * kC * kC * 9) + align256(8 * 3 * 64 * size_t(batch));
}

// Forward for a batch: acts (nullable for batch 1 with tmp0/tmp1 ping-pong buffers) keeps the
// outputs of layers 1..5; scale (batch floats) receives 1/RMS of each input; wr receives the
// reordered weights (BSC_NET_PARAMS floats; pass reordered = true if it already holds them).
hipError_t net_forward_impl(int n_u, int n_v, int batch, const float *w, const float *in, float *out, float *acts,
                            float *tmp0, float *tmp1, float *scale, float *wr, bool reordered, hipStream_t st) {
    const size_t n = size_t(n_u) * n_v;
    if (!reordered) reorder_all(w, wr, 0, st);
    k_rms<<<batch, 256, 0, st>>>(in, int(n), scale);
    float *A[5];
    for (int l = 0; l < 5; ++l) A[l] = acts ? acts + size_t(l) * batch * kC * n : ((l & 1) ? tmp1 : tmp0);
    conv<3, 32, 1>(n_u, n_v, batch, in, wr + layer_offset(0), A[0], nullptr, scale, st);
    for (int l = 1; l < 5; ++l) conv<32, 32, 1>(n_u, n_v, batch, A[l - 1], wr + layer_offset(l), A[l], nullptr, nullptr, st);
    conv<32, 3, 0>(n_u, n_v, batch, A[4], wr + layer_offset(5), out, nullptr, nullptr, st);
    return hipGetLastError();
}

hipError_t net_backward(int n_u, int n_v, int batch, const float *w, const float *in, const float *acts,
                        const float *dout, float *dw, float *din, void *scratch, hipStream_t st) {
    const size_t n = size_t(n_u) * n_v;
    const int tiles = ((n_u + kT - 1) / kT) * ((n_v + kT - 1) / kT);
    NetScratch s = carve(scratch, n_u, n_v, batch);
    k_rms<<<batch, 256, 0, st>>>(in, int(n), s.scale);
    reorder_all(w, s.wt, 1, st);
    const dim3 g = conv_grid(n_u, n_v, batch);
    const float *A[5];
    for (int l = 0; l < 5; ++l) A[l] = acts + size_t(l) * batch * kC * n;
    // layer 6 (32 -> 3, linear): dZ6 = dout
    const float *dz = dout;
    float *bufs[2] = {s.dz0, s.dz1};
    int nb = 0;
    for (int l = kLayers - 1; l >= 0; --l) {
        const float *X = l == 0 ? in : A[l - 1];
        const float *xs = l == 0 ? s.scale : nullptr;
        const int len = kCin[l] * kCout[l] * 9;
        if (l == 0) k_dw_tile<3, 32><<<g, kT * kT, 0, st>>>(n_u, n_v, X, dz, xs, s.part);
        else if (l == kLayers - 1) k_dw_tile<32, 3><<<g, kT * kT, 0, st>>>(n_u, n_v, X, dz, xs, s.part);
        else k_dw_tile<32, 32><<<g, kT * kT, 0, st>>>(n_u, n_v, X, dz, xs, s.part);
        k_dw_reduce<<<(len + 255) / 256, 256, 0, st>>>(s.part, tiles * batch, len, dw + layer_offset(l));
        if (l > 0) {
            // dZ_{l-1} = (W_l^T conv dZ_l) * LeakyReLU'(A_{l-1})
            float *dst = bufs[nb];
            nb ^= 1;
            if (l == kLayers - 1) conv<3, 32, 2>(n_u, n_v, batch, dz, s.wt + layer_offset(l), dst, A[l - 1], nullptr, st);
            else conv<32, 32, 2>(n_u, n_v, batch, dz, s.wt + layer_offset(l), dst, A[l - 1], nullptr, st);
            dz = dst;
        } else if (din) {
            // gradient with respect to the normalised input
            conv<32, 3, 0>(n_u, n_v, batch, dz, s.wt + layer_offset(0), din, nullptr, nullptr, st);
        }
    }
    return hipGetLastError();
}

hipError_t net_adam(int n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2, float eps, int t,
                    hipStream_t st) {
    const float c1 = 1.0f - powf(b1, float(t)), c2 = 1.0f - powf(b2, float(t));
    k_adam<<<(n + 255) / 256, 256, 0, st>>>(n, p, g, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t net_loss(int n_cp, int batch, const float *in, const float *pred, const float *tgt, float *loss, float *dpred,
                    double *part, hipStream_t st) {
    constexpr int nb = 64;
    k_loss_part<<<dim3(nb, batch), 256, 0, st>>>(n_cp, pred, tgt, in, part, nb);
    k_loss_grad<<<dim3(nb, batch), 256, 0, st>>>(n_cp, batch, pred, tgt, in, part, nb, loss, dpred);
    return hipGetLastError();
}

// Scratch of bsc_net_backward_noalloc: one static array per device, reached from host code only
// through the address hipGetSymbolAddress returns on that device (the array's name is a host-side
// stand-in there). Looked up once per device, under a lock, the first time a context on that
// device calls the entry point.
static __device__ __align__(256) unsigned char scratch[BSC_NET_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

bsc_status static_scratch_address(bsc_ctx *c, void **out) {
    if (c->device < 0 || c->device >= kMaxDevices) return fail(c, BSC_E_INVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[c->device]) {
        int prev = 0;
        bsc_status st = hip_check(c, hipGetDevice(&prev), "hipGetDevice");
        if (st != BSC_OK) return st;
        if (prev != c->device) {
            st = hip_check(c, hipSetDevice(c->device), "hipSetDevice");
            if (st != BSC_OK) return st;
        }
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != c->device) (void)hipSetDevice(prev);
        st = hip_check(c, e, "hipGetSymbolAddress(scratch)");
        if (st != BSC_OK) return st;
        if (!p) return fail(c, BSC_E_HIP, "hipGetSymbolAddress(scratch) returned a null address");
        g_scratch_ptr[c->device] = p;
    }
    *out = g_scratch_ptr[c->device];
    return BSC_OK;
}

}  // namespace bsc

using namespace bsc;

extern "C" {

bsc_status bsc_warmstart_load(bsc_ctx *c, const float *d_weights, int32_t n_params) {
    if (!c) return BSC_E_INVAL;
    if (!c->ws) return fail(c, BSC_E_STATE, "no workspace bound");
    if (!d_weights || n_params != BSC_NET_PARAMS) return fail(c, BSC_E_INVAL, "expected BSC_NET_PARAMS weights");
    bsc_status st = hip_check(c, hipMemcpyAsync(c->buf.net_w, d_weights, 4 * size_t(BSC_NET_PARAMS), hipMemcpyDeviceToDevice, c->stream), "load weights");
    if (st != BSC_OK) return st;
    reorder_all(c->buf.net_w, c->buf.net_w_fwd, 0, c->stream);
    st = hip_check(c, hipGetLastError(), "reorder weights");
    if (st != BSC_OK) return st;
    st = hip_check(c, hipStreamSynchronize(c->stream), "load weights");
    if (st == BSC_OK) c->net_loaded = true;
    return st;
}

bsc_status bsc_net_forward(bsc_ctx *c, int32_t batch, const float *d_weights, const float *d_in, float *d_out, float *d_acts) {
    if (!c) return BSC_E_INVAL;
    if (!c->ws) return fail(c, BSC_E_STATE, "no workspace bound");
    if (batch < 1 || batch > 1024 || !d_weights || !d_in || !d_out) return fail(c, BSC_E_INVAL, "bad arguments");
    if (batch > 1 && !d_acts) return fail(c, BSC_E_INVAL, "batch > 1 needs d_acts");
    return hip_check(c, net_forward_impl(c->n_u, c->n_v, batch, d_weights, d_in, d_out, d_acts, c->buf.net_act0,
                                         c->buf.net_act1, c->buf.net_scale, c->buf.net_wr, false, c->stream), "net forward");
}

bsc_status bsc_net_scratch_size(const bsc_ctx *c, int32_t batch, size_t *bytes) {
    if (!c || !bytes || batch < 1 || batch > 1024) return BSC_E_INVAL;
    *bytes = net_scratch_bytes(c->n_u, c->n_v, batch);
    return BSC_OK;
}

bsc_status bsc_net_backward(bsc_ctx *c, int32_t batch, const float *d_weights, const float *d_in, const float *d_acts,
                            const float *d_dout, float *d_dweights, float *d_din, void *d_scratch) {
    if (!c) return BSC_E_INVAL;
    if (!c->ws) return fail(c, BSC_E_STATE, "no workspace bound");
    if (batch < 1 || batch > 1024 || !d_weights || !d_in || !d_acts || !d_dout || !d_dweights || !d_scratch)
        return fail(c, BSC_E_INVAL, "bad arguments");
    return hip_check(c, net_backward(c->n_u, c->n_v, batch, d_weights, d_in, d_acts, d_dout, d_dweights, d_din, d_scratch,
                                     c->stream), "net backward");
}

bsc_status bsc_net_backward_noalloc(bsc_ctx *c, int32_t batch, const float *d_weights, const float *d_in,
                                    const float *d_acts, const float *d_dout, float *d_dweights, float *d_din) {
    if (!c) return BSC_E_INVAL;
    if (!c->ws) return fail(c, BSC_E_STATE, "no workspace bound");
    if (batch < 1 || batch > 1024 || !d_weights || !d_in || !d_acts || !d_dout || !d_dweights)
        return fail(c, BSC_E_INVAL, "bad arguments");
    const size_t need = net_scratch_bytes(c->n_u, c->n_v, batch);
    if (need > size_t(BSC_NET_NOALLOC_SCRATCH_BYTES))
        return fail(c, BSC_E_INVAL, "bsc_net_backward_noalloc: this grid and batch need " + std::to_string(need) +
                                        " scratch bytes, more than the static " +
                                        std::to_string(size_t(BSC_NET_NOALLOC_SCRATCH_BYTES)) +
                                        "; use bsc_net_backward with a caller workspace");
    void *base = nullptr;
    bsc_status st = static_scratch_address(c, &base);
    if (st != BSC_OK) return st;
    return hip_check(c, net_backward(c->n_u, c->n_v, batch, d_weights, d_in, d_acts, d_dout, d_dweights, d_din, base,
                                     c->stream), "net backward (static scratch)");
}

bsc_status bsc_net_loss(bsc_ctx *c, int32_t batch, const float *d_in, const float *d_pred, const float *d_target,
                        float *d_loss, float *d_dpred) {
    if (!c) return BSC_E_INVAL;
    if (!c->ws) return fail(c, BSC_E_STATE, "no workspace bound");
    if (batch < 1 || batch > 1024 || !d_in || !d_pred || !d_target || !d_loss || !d_dpred) return fail(c, BSC_E_INVAL, "bad arguments");
    return hip_check(c, net_loss(c->n_cp, batch, d_in, d_pred, d_target, d_loss, d_dpred, c->buf.net_lpart, c->stream), "net loss");
}

bsc_status bsc_adam_step(bsc_ctx *c, int32_t n, float *d_param, const float *d_grad, float *d_m, float *d_v, float lr,
                         float beta1, float beta2, float eps, int32_t t) {
    if (!c) return BSC_E_INVAL;
    if (n < 1 || t < 1 || !d_param || !d_grad || !d_m || !d_v) return fail(c, BSC_E_INVAL, "bad arguments");
    return hip_check(c, net_adam(n, d_param, d_grad, d_m, d_v, lr, beta1, beta2, eps, t, c->stream), "adam");
}

}  // extern "C"
