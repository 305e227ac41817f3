// Learned initial guess for Newton: a small 3x3 convolutional network on the
// interior vertex grid (NHWC: batch, y, x, channel), trained on solutions
// the solver itself produces.  The paper has no learned component; this is
// the project's own design.
//
//   Z_l = conv3x3(A_{l-1}, W_l) + b_l,  A_l = max(Z_l, 0),  O = Z_L,
//   U[.., k] = env(y, x) * oscale[k] * O[.., k]
//   loss = mean (env O - T / oscale)^2,  Adam on FP32 master weights.
//
// Both convolution passes that have the shape of a convolution (forward, and
// the gradient with respect to a layer input, a convolution with the kernel
// flipped and its channel axes swapped) run on the matrix cores as implicit
// GEMMs: BF16 operands (16x16x32 MFMA), FP32 accumulation.  The weight
// gradient is a reduction over all pixels of products of two BF16 tensors;
// it runs on the vector units in FP32 over pixel chunks, with the chunk
// partial sums added in a fixed order.
#include "common.hpp"

#include <algorithm>
#include <cmath>

typedef __bf16 nn_bf8 __attribute__((ext_vector_type(8)));
typedef float nn_f4 __attribute__((ext_vector_type(4)));

struct sg_nn {
    int device = 0;
    int H = 0, W = 0, max_batch = 0, nl = 0;
    std::vector<int> ci, co;          // real channel counts per layer
    std::vector<int> cip, cop;        // padded: inputs to 8, outputs to 16
    std::vector<int64_t> woff, boff;  // offsets in the flat parameter vector
    int64_t nparam = 0;
    int t = 0;                        // Adam steps taken
    sg::DevBuf<float> p, g, m, v;     // master parameters, gradient, Adam moments
    std::vector<sg::DevBuf<uint16_t>> wf, wb;   // packed BF16 kernels: forward, input gradient
    std::vector<sg::DevBuf<float>> bias;        // padded biases
    sg::DevBuf<uint16_t> x16;                   // [B,H,W,cip0]
    std::vector<sg::DevBuf<uint16_t>> act;      // A_1 .. A_{L-1}
    sg::DevBuf<float> out;                      // O [B,H,W,cop_last]
    sg::DevBuf<uint16_t> dz0, dz1;              // gradients w.r.t. Z (ping-pong)
    sg::DevBuf<float> wpart, bpart;             // weight-gradient chunk partials
    sg::DevBuf<double> lpart;                   // loss partials
    sg::DevBuf<float> env, oscale;
    bool have_map = false;
};

namespace sg {
namespace {

constexpr int kNT = 256;
constexpr int kChunkPix = 1024;      // pixels per weight-gradient work-group
constexpr int kSubPix = 64;          // pixels staged in LDS at a time

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------- conv
// One wave computes 32 pixels x NT*16 output channels; K = 9 taps x cinp
// input channels in chunks of 32 (lane group g holds the 8 consecutive
// channels k0 = 32c + 8g of one tap).  Zero padding by bounds checks.
template <int NT>
__global__ __launch_bounds__(kNT) void conv_mfma_kernel(
    int npix, int H, int W, int cinp, int nchunk, const uint16_t* __restrict__ in,
    const uint16_t* __restrict__ wk, const float* __restrict__ bias, int relu,
    const uint16_t* __restrict__ mask, uint16_t* __restrict__ out16, float* __restrict__ out32) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int base = (blockIdx.x * (kNT / 64) + wave) * 32;
    if (base >= npix) return;
    const int HW = H * W;
    int pb[2], py[2], px[2];
    bool pv[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        const int p = base + 16 * t + r;
        pv[t] = p < npix;
        const int pp = pv[t] ? p : 0;
        pb[t] = pp / HW;
        const int rem = pp - pb[t] * HW;
        py[t] = rem / W;
        px[t] = rem - py[t] * W;
    }
    nn_f4 acc[2][NT];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[t][j] = nn_f4{0.f, 0.f, 0.f, 0.f};
    for (int c = 0; c < nchunk; ++c) {
        const int k0 = 32 * c + 8 * g;
        const int tap = k0 / cinp, c0 = k0 - tap * cinp;
        nn_bf8 b[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const uint4 q = *reinterpret_cast<const uint4*>(wk + ((size_t)(c * NT * 16 + j * 16 + r)) * 32 + 8 * g);
            __builtin_memcpy(&b[j], &q, 16);
        }
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            uint4 q = make_uint4(0u, 0u, 0u, 0u);
            if (pv[t] && tap < 9) {
                const int yy = py[t] + tap / 3 - 1, xx = px[t] + tap % 3 - 1;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                    q = *reinterpret_cast<const uint4*>(in + ((size_t)(pb[t] * HW + yy * W + xx)) * cinp + c0);
            }
            nn_bf8 a;
            __builtin_memcpy(&a, &q, 16);
#pragma unroll
            for (int j = 0; j < NT; ++j)
                acc[t][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], acc[t][j], 0, 0, 0);
        }
    }
    constexpr int C = NT * 16;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int p = base + 16 * t + 4 * g + v;
                if (p >= npix) continue;
                const int ch = 16 * j + r;
                float val = acc[t][j][v];
                if (bias) val += bias[ch];
                if (relu) val = fmaxf(val, 0.f);
                if (mask) {
                    const uint16_t mb = mask[(size_t)p * C + ch];
                    if ((mb & 0x8000u) || !(mb & 0x7fffu)) val = 0.f;   // activation <= 0
                }
                if (out16) out16[(size_t)p * C + ch] = f2bf(val);
                if (out32) out32[(size_t)p * C + ch] = val;
            }
}

// Packed kernels.  Forward: K row k = 32c + kk of chunk c is (tap, ci) =
// (k / cinp, k % cinp); entry [c][o][kk] = W[tap][ci][o].  Input gradient:
// input channels are the layer's outputs, tap' = 8 - tap (flipped kernel).
__global__ void pack_kernel(int nchunk, int cop_out, int cinp_in, int n_in, int n_out, int flip,
                            const float* __restrict__ Wt, int w_ci, int w_co,
                            uint16_t* __restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)nchunk * cop_out * 32;
    if (idx >= total) return;
    const int kk = (int)(idx % 32);
    const int o = (int)((idx / 32) % cop_out);
    const int c = (int)(idx / (32 * (int64_t)cop_out));
    const int k = 32 * c + kk;
    const int tap = k / cinp_in, i = k - tap * cinp_in;
    float val = 0.f;
    if (tap < 9 && i < n_in && o < n_out) {
        // forward: (i, o) = (ci, co); input gradient: (i, o) = (co, ci)
        val = flip ? Wt[((size_t)(8 - tap) * w_ci + o) * w_co + i] : Wt[((size_t)tap * w_ci + i) * w_co + o];
    }
    out[idx] = f2bf(val);
}

__global__ void pad_bias_kernel(int n, int np, const float* __restrict__ b, float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np) out[i] = i < n ? b[i] : 0.f;
}

__global__ void input_kernel(int64_t npix, int cin, int cinp, const double* __restrict__ X,
                             uint16_t* __restrict__ x16) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= npix * cinp) return;
    const int64_t p = idx / cinp;
    const int c = (int)(idx - p * cinp);
    x16[idx] = c < cin ? f2bf((float)X[p * cin + c]) : (uint16_t)0;
}

// dO = 2 env (env O - T / oscale) / count (zero on padded channels); block
// partial sums of the squared error in FP64.
__global__ __launch_bounds__(kNT) void loss_kernel(int64_t npix, int HW, int cout, int cop,
                                                   const float* __restrict__ O,
                                                   const double* __restrict__ T,
                                                   const float* __restrict__ env,
                                                   const float* __restrict__ osc, double inv_count,
                                                   uint16_t* __restrict__ dO, double* __restrict__ part) {
    __shared__ double red[kNT];
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e2 = 0.0;
    if (idx < npix * cop) {
        const int64_t p = idx / cop;
        const int k = (int)(idx - p * cop);
        float gr = 0.f;
        if (k < cout) {
            const double e = env[p % HW];
            const double E = e * (double)O[idx] - T[p * cout + k] / (double)osc[k];
            e2 = E * E;
            gr = (float)(2.0 * e * E * inv_count);
        }
        dO[idx] = f2bf(gr);
    }
    red[threadIdx.x] = e2;
    __syncthreads();
    for (int o = kNT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sum_kernel(int n, const double* __restrict__ part, double* __restrict__ out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += part[i];
        out[0] = s;
    }
}

// Weight gradient partials over one chunk of pixels for one tap: each thread
// owns a 4 x 4 block of (input channel, output channel); the chunk's shifted
// inputs and output gradients are staged in LDS kSubPix pixels at a time.
// The tap-4 (centre) work-groups also sum the output gradient for the bias.
__global__ __launch_bounds__(kNT) void wgrad_kernel(int64_t npix, int H, int W, int cinp, int cin,
                                                    int cout, int cop, const uint16_t* __restrict__ in,
                                                    const uint16_t* __restrict__ dz,
                                                    float* __restrict__ wpart, float* __restrict__ bpart) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    uint16_t* sin = reinterpret_cast<uint16_t*>(smem_raw);          // [kSubPix][cinp]
    uint16_t* sdz = sin + kSubPix * cinp;                            // [kSubPix][cop]
    const int chunk = blockIdx.x, tap = blockIdx.y;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    const int nci4 = (cin + 3) / 4, nco4 = (cout + 3) / 4;
    const int tid = threadIdx.x;
    const bool active = tid < nci4 * nco4;
    const int i4 = active ? tid / nco4 : 0, o4 = active ? tid - (tid / nco4) * nco4 : 0;
    float acc[4][4] = {};
    float bacc[4] = {0.f, 0.f, 0.f, 0.f};
    const int HW = H * W;
    const int64_t p0 = (int64_t)chunk * kChunkPix;
    for (int s0 = 0; s0 < kChunkPix; s0 += kSubPix) {
        __syncthreads();
        for (int q = tid; q < kSubPix * cinp; q += kNT) {
            const int pl = q / cinp, c = q - pl * cinp;
            const int64_t p = p0 + s0 + pl;
            uint16_t val = 0;
            if (p < npix) {
                const int b = (int)(p / HW);
                const int rem = (int)(p - (int64_t)b * HW);
                const int yy = rem / W + dy, xx = rem % W + dx;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                    val = in[((int64_t)b * HW + yy * W + xx) * cinp + c];
            }
            sin[q] = val;
        }
        for (int q = tid; q < kSubPix * cop; q += kNT) {
            const int pl = q / cop;
            const int64_t p = p0 + s0 + pl;
            sdz[q] = p < npix ? dz[p * cop + (q - pl * cop)] : (uint16_t)0;
        }
        __syncthreads();
        if (active) {
            for (int pl = 0; pl < kSubPix; ++pl) {
                float a[4], d[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int ci = 4 * i4 + u, co = 4 * o4 + u;
                    a[u] = ci < cinp ? bf2f(sin[pl * cinp + ci]) : 0.f;
                    d[u] = co < cop ? bf2f(sdz[pl * cop + co]) : 0.f;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int w = 0; w < 4; ++w) acc[u][w] = fmaf(a[u], d[w], acc[u][w]);
                if (tap == 4 && i4 == 0)
#pragma unroll
                    for (int w = 0; w < 4; ++w) bacc[w] += d[w];
            }
        }
    }
    if (!active) return;
    float* wp = wpart + ((size_t)chunk * 9 + tap) * cin * cout;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int ci = 4 * i4 + u, co = 4 * o4 + w;
            if (ci < cin && co < cout) wp[(size_t)ci * cout + co] = acc[u][w];
        }
    if (tap == 4 && i4 == 0)
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int co = 4 * o4 + w;
            if (co < cout) bpart[(size_t)chunk * cout + co] = bacc[w];
        }
}

// g[W] = sum over chunks of the partials (fixed order); same for the bias.
__global__ void wreduce_kernel(int nchunks, int nw, int nb, const float* __restrict__ wpart,
                               const float* __restrict__ bpart, float* __restrict__ gw,
                               float* __restrict__ gb) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < nw) {
        // partial layout [chunk][tap][ci][co]; gradient layout [tap][ci][co]: same inner order
        float s = 0.f;
        for (int c = 0; c < nchunks; ++c) s += wpart[(size_t)c * nw + idx];
        gw[idx] = s;
    } else if (idx < nw + nb) {
        const int o = idx - nw;
        float s = 0.f;
        for (int c = 0; c < nchunks; ++c) s += bpart[(size_t)c * nb + o];
        gb[o] = s;
    }
}

__global__ void adam_kernel(int64_t n, float lr, float b1, float b2, float eps, float c1, float c2,
                            float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void predict_kernel(int64_t npix, int HW, int cout, int cop, const float* __restrict__ O,
                               const float* __restrict__ env, const float* __restrict__ osc,
                               double* __restrict__ U) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= npix * cout) return;
    const int64_t p = idx / cout;
    const int k = (int)(idx - p * cout);
    U[idx] = (double)env[p % HW] * (double)osc[k] * (double)O[p * cop + k];
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kNT - 1) / kNT); }
inline int pad_to(int v, int m) { return (v + m - 1) / m * m; }

void launch_conv(int NT, int npix, int H, int W, int cinp, const uint16_t* in, const uint16_t* wk,
                 const float* bias, int relu, const uint16_t* mask, uint16_t* o16, float* o32,
                 hipStream_t s) {
    const int nchunk = (9 * cinp + 31) / 32;
    const unsigned grid = (unsigned)((npix + 32 * (kNT / 64) - 1) / (32 * (kNT / 64)));
    switch (NT) {
        case 1: conv_mfma_kernel<1><<<grid, kNT, 0, s>>>(npix, H, W, cinp, nchunk, in, wk, bias, relu, mask, o16, o32); break;
        case 2: conv_mfma_kernel<2><<<grid, kNT, 0, s>>>(npix, H, W, cinp, nchunk, in, wk, bias, relu, mask, o16, o32); break;
        case 3: conv_mfma_kernel<3><<<grid, kNT, 0, s>>>(npix, H, W, cinp, nchunk, in, wk, bias, relu, mask, o16, o32); break;
        case 4: conv_mfma_kernel<4><<<grid, kNT, 0, s>>>(npix, H, W, cinp, nchunk, in, wk, bias, relu, mask, o16, o32); break;
        default: SG_THROW(SG_ERR_UNSUPPORTED, "conv with %d output tiles", NT);
    }
    HIP_LAUNCH_OK();
}

void pack_weights(sg_nn* nn, hipStream_t s) {
    for (int l = 0; l < nn->nl; ++l) {
        const float* Wt = nn->p.p + nn->woff[l];
        const int nchf = (9 * nn->cip[l] + 31) / 32;
        int64_t tot = (int64_t)nchf * nn->cop[l] * 32;
        pack_kernel<<<blocks_for(tot), kNT, 0, s>>>(nchf, nn->cop[l], nn->cip[l], nn->ci[l], nn->co[l],
                                                     0, Wt, nn->ci[l], nn->co[l], nn->wf[l].p);
        HIP_LAUNCH_OK();
        if (l > 0) {
            const int cin_b = nn->cop[l];              // input gradient: inputs are dZ_l
            const int cout_b = pad_to(nn->ci[l], 16);
            const int nchb = (9 * cin_b + 31) / 32;
            tot = (int64_t)nchb * cout_b * 32;
            pack_kernel<<<blocks_for(tot), kNT, 0, s>>>(nchb, cout_b, cin_b, nn->co[l], nn->ci[l], 1,
                                                         Wt, nn->ci[l], nn->co[l], nn->wb[l].p);
            HIP_LAUNCH_OK();
        }
        pad_bias_kernel<<<1, 128, 0, s>>>(nn->co[l], nn->cop[l], nn->p.p + nn->boff[l], nn->bias[l].p);
        HIP_LAUNCH_OK();
    }
}

// Forward pass of B samples: X [B,H,W,ci0] FP64 -> out (FP32, padded).
void nn_forward_core(sg_nn* nn, const double* X, int B, hipStream_t s) {
    const int64_t npix = (int64_t)B * nn->H * nn->W;
    input_kernel<<<blocks_for(npix * nn->cip[0]), kNT, 0, s>>>(npix, nn->ci[0], nn->cip[0], X, nn->x16.p);
    HIP_LAUNCH_OK();
    const uint16_t* cur = nn->x16.p;
    for (int l = 0; l < nn->nl; ++l) {
        const bool last = l + 1 == nn->nl;
        launch_conv(nn->cop[l] / 16, (int)npix, nn->H, nn->W, nn->cip[l], cur, nn->wf[l].p,
                    nn->bias[l].p, last ? 0 : 1, nullptr, last ? nullptr : nn->act[l].p,
                    last ? nn->out.p : nullptr, s);
        if (!last) cur = nn->act[l].p;
    }
}

// Loss and gradient (into nn->g) for B samples.
double nn_backward_core(sg_nn* nn, const double* X, const double* T, int B, hipStream_t s) {
    SG_REQUIRE(nn->have_map, "output map (env, oscale) not set");
    nn_forward_core(nn, X, B, s);
    const int64_t npix = (int64_t)B * nn->H * nn->W;
    const int L = nn->nl;
    const int HW = nn->H * nn->W;
    const double inv_count = 1.0 / ((double)npix * nn->co[L - 1]);
    const unsigned lb = blocks_for(npix * nn->cop[L - 1]);
    SG_REQUIRE((size_t)lb + 1 <= nn->lpart.n, "loss partial buffer too small");
    loss_kernel<<<lb, kNT, 0, s>>>(npix, HW, nn->co[L - 1], nn->cop[L - 1], nn->out.p, T,
                                   nn->env.p, nn->oscale.p, inv_count, nn->dz0.p, nn->lpart.p);
    HIP_LAUNCH_OK();
    sum_kernel<<<1, 1, 0, s>>>((int)lb, nn->lpart.p, nn->lpart.p + lb);
    HIP_LAUNCH_OK();
    uint16_t* dz = nn->dz0.p;
    uint16_t* dn = nn->dz1.p;
    const int nchunks = (int)((npix + kChunkPix - 1) / kChunkPix);
    for (int l = L - 1; l >= 0; --l) {
        const uint16_t* in = l == 0 ? nn->x16.p : nn->act[l - 1].p;
        const int cinp_in = l == 0 ? nn->cip[0] : nn->cop[l - 1];
        const size_t lds = (size_t)kSubPix * (cinp_in + nn->cop[l]) * sizeof(uint16_t);
        dim3 grid((unsigned)nchunks, 9);
        wgrad_kernel<<<grid, kNT, lds, s>>>(npix, nn->H, nn->W, cinp_in, nn->ci[l], nn->co[l],
                                            nn->cop[l], in, dz, nn->wpart.p, nn->bpart.p);
        HIP_LAUNCH_OK();
        const int nw = 9 * nn->ci[l] * nn->co[l];
        wreduce_kernel<<<blocks_for(nw + nn->co[l]), kNT, 0, s>>>(
            nchunks, nw, nn->co[l], nn->wpart.p, nn->bpart.p, nn->g.p + nn->woff[l],
            nn->g.p + nn->boff[l]);
        HIP_LAUNCH_OK();
        if (l > 0) {
            // dA_{l-1} = conv(dZ_l, flipped W_l), then dZ_{l-1} = dA_{l-1} * (A_{l-1} > 0)
            launch_conv(pad_to(nn->ci[l], 16) / 16, (int)npix, nn->H, nn->W, nn->cop[l], dz,
                        nn->wb[l].p, nullptr, 0, nn->act[l - 1].p, dn, nullptr, s);
            std::swap(dz, dn);
        }
    }
    double sse = 0.0;
    HIP_OK(hipMemcpyAsync(&sse, nn->lpart.p + lb, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return sse * inv_count;
}

// Network inputs of a draw at npts points: [c0, g_1 .. g_M] with the
// log-normal mean c0 = exp(g0 + |g|^2 / 2) (Eq. inputlogn).
__global__ void input_fields_kernel(int npts, int M, const double* __restrict__ g0,
                                    const double* __restrict__ g, double* __restrict__ X) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npts) return;
    double s = 0.0;
    for (int m = 0; m < M; ++m) {
        const double v = g[(size_t)m * npts + p];
        s = fma(v, v, s);
        X[(size_t)p * (M + 1) + 1 + m] = v;
    }
    X[(size_t)p * (M + 1)] = exp(g0[p] + 0.5 * s);
}

// One work-group: fixed-order block reduction of n values of f(i) (sum or max).
template <bool MAX, class F>
__device__ double block_reduce(int64_t n, F f) {
    __shared__ double sh[kNT];
    double a = MAX ? -INFINITY : 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kNT) {
        const double v = f(i);
        a = MAX ? fmax(a, v) : a + v;
    }
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int w = kNT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            sh[threadIdx.x] = MAX ? fmax(sh[threadIdx.x], sh[threadIdx.x + w])
                                  : sh[threadIdx.x] + sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// env = shape / max(shape) (FP32) and its mean square; one work-group.
__global__ void envelope_kernel(int HW, const double* __restrict__ shape, float* __restrict__ env,
                                double* __restrict__ env_ms) {
    const double mx = block_reduce<true>(HW, [&](int64_t i) { return shape[i]; });
    for (int i = threadIdx.x; i < HW; i += kNT) env[i] = (float)(shape[i] / mx);
    const double ms = block_reduce<false>(HW, [&](int64_t i) {
        const double e = shape[i] / mx;
        return e * e;
    });
    if (threadIdx.x == 0) env_ms[0] = ms / HW;
}

// oscale[k] = max(RMS of mode k over the B samples and all pixels, 1e-30) /
// RMS(env); one work-group per mode.
__global__ void mode_scale_kernel(int64_t npix, int cout, const double* __restrict__ T,
                                  const double* __restrict__ env_ms, float* __restrict__ oscale) {
    const int k = blockIdx.x;
    const double ss = block_reduce<false>(npix, [&](int64_t p) {
        const double t = T[p * cout + k];
        return t * t;
    });
    if (threadIdx.x == 0)
        oscale[k] = (float)(fmax(sqrt(ss / (double)npix), 1e-30) / sqrt(env_ms[0]));
}

}  // namespace
}  // namespace sg

using namespace sg;

extern "C" {

int nn_input_fields(int npts, int M, const double* g0, const double* g, double* X, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(npts >= 1 && M >= 0 && M <= 16, "bad sizes (npts %d, M %d)", npts, M);
        SG_REQUIRE(g0 && X && (M == 0 || g), "null argument");
        input_fields_kernel<<<blocks_for(npts), kNT, 0, as_stream(stream)>>>(npts, M, g0, g, X);
        HIP_LAUNCH_OK();
        return SG_OK;
    });
}

int nn_fit_output_map(sg_nn* nn, const double* shape, const double* T, int B, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(nn && shape && T, "null argument");
        SG_REQUIRE(B >= 1, "B must be >= 1");
        check_device(nn->device);
        hipStream_t s = as_stream(stream);
        const int HW = nn->H * nn->W, cout = nn->co[nn->nl - 1];
        DevBuf<double> ms(1);
        envelope_kernel<<<1, kNT, 0, s>>>(HW, shape, nn->env.p, ms.p);
        HIP_LAUNCH_OK();
        mode_scale_kernel<<<cout, kNT, 0, s>>>((int64_t)B * HW, cout, T, ms.p, nn->oscale.p);
        HIP_LAUNCH_OK();
        HIP_OK(hipStreamSynchronize(s));
        nn->have_map = true;
        return SG_OK;
    });
}


int nn_create(int n_layers, const int32_t* channels, int H, int W, int max_batch, sg_nn** out) {
    return guarded([&]() -> int {
        SG_REQUIRE(out && channels, "null argument");
        SG_REQUIRE(n_layers >= 1 && n_layers <= 16, "n_layers=%d outside [1,16]", n_layers);
        SG_REQUIRE(H >= 1 && W >= 1 && max_batch >= 1, "bad grid or batch");
        SG_REQUIRE((int64_t)max_batch * H * W < (int64_t)INT32_MAX / 64, "batch too large");
        auto nn = std::make_unique<sg_nn>();
        nn->device = current_device();
        nn->H = H; nn->W = W; nn->max_batch = max_batch; nn->nl = n_layers;
        int64_t q = 0;
        for (int l = 0; l < n_layers; ++l) {
            const int a = channels[l], b = channels[l + 1];
            SG_REQUIRE(a >= 1 && b >= 1 && a <= 64 && b <= 64, "channels must be in [1,64]");
            nn->ci.push_back(a);
            nn->co.push_back(b);
            nn->cop.push_back(pad_to(b, 16));
            nn->woff.push_back(q);
            q += 9LL * a * b;
            nn->boff.push_back(q);
            q += b;
        }
        for (int l = 0; l < n_layers; ++l)
            nn->cip.push_back(l == 0 ? pad_to(nn->ci[0], 8) : nn->cop[l - 1]);
        nn->nparam = q;
        nn->p.alloc(q); nn->g.alloc(q); nn->m.alloc(q); nn->v.alloc(q);
        HIP_OK(hipMemset(nn->p.p, 0, q * 4));
        HIP_OK(hipMemset(nn->g.p, 0, q * 4));
        HIP_OK(hipMemset(nn->m.p, 0, q * 4));
        HIP_OK(hipMemset(nn->v.p, 0, q * 4));
        const int64_t npix = (int64_t)max_batch * H * W;
        int maxc = 0;
        for (int l = 0; l < n_layers; ++l) {
            nn->wf.emplace_back((size_t)((9 * nn->cip[l] + 31) / 32) * nn->cop[l] * 32);
            if (l > 0)
                nn->wb.emplace_back((size_t)((9 * nn->cop[l] + 31) / 32) * pad_to(nn->ci[l], 16) * 32);
            else
                nn->wb.emplace_back();
            nn->bias.emplace_back((size_t)nn->cop[l]);
            if (l + 1 < n_layers) nn->act.emplace_back((size_t)(npix * nn->cop[l]));
            maxc = std::max(maxc, std::max(nn->cop[l], pad_to(nn->ci[l], 16)));
        }
        nn->x16.alloc((size_t)(npix * nn->cip[0]));
        nn->out.alloc((size_t)(npix * nn->cop[n_layers - 1]));
        nn->dz0.alloc((size_t)(npix * maxc));
        nn->dz1.alloc((size_t)(npix * maxc));
        const int64_t nchunks = (npix + kChunkPix - 1) / kChunkPix;
        int64_t wmax = 0, bmax = 0;
        for (int l = 0; l < n_layers; ++l) {
            wmax = std::max<int64_t>(wmax, 9LL * nn->ci[l] * nn->co[l]);
            bmax = std::max<int64_t>(bmax, nn->co[l]);
        }
        nn->wpart.alloc((size_t)(nchunks * wmax));
        nn->bpart.alloc((size_t)(nchunks * bmax));
        nn->lpart.alloc((size_t)(blocks_for(npix * nn->cop[n_layers - 1]) + 1));
        nn->env.alloc((size_t)H * W);
        nn->oscale.alloc((size_t)nn->co[n_layers - 1]);
        pack_weights(nn.get(), nullptr);
        HIP_OK(hipDeviceSynchronize());
        *out = nn.release();
        return SG_OK;
    });
}

int64_t nn_param_count(const sg_nn* nn) { return nn ? nn->nparam : 0; }

int nn_set_params(sg_nn* nn, const float* params) {
    return guarded([&]() -> int {
        SG_REQUIRE(nn && params, "null argument");
        check_device(nn->device);
        nn->p.upload(params, nn->nparam, nullptr);
        HIP_OK(hipMemset(nn->m.p, 0, nn->nparam * 4));
        HIP_OK(hipMemset(nn->v.p, 0, nn->nparam * 4));
        nn->t = 0;
        pack_weights(nn, nullptr);
        HIP_OK(hipDeviceSynchronize());
        return SG_OK;
    });
}

int nn_get_params(const sg_nn* nn, float* params, float* grads) {
    return guarded([&]() -> int {
        SG_REQUIRE(nn != nullptr, "nn is NULL");
        check_device(nn->device);
        if (params) nn->p.download(params, nn->nparam, nullptr);
        if (grads) nn->g.download(grads, nn->nparam, nullptr);
        HIP_OK(hipDeviceSynchronize());
        return SG_OK;
    });
}

int nn_set_output_map(sg_nn* nn, const float* env, const float* oscale) {
    return guarded([&]() -> int {
        SG_REQUIRE(nn && env && oscale, "null argument");
        check_device(nn->device);
        nn->env.upload(env, (size_t)nn->H * nn->W, nullptr);
        nn->oscale.upload(oscale, nn->co[nn->nl - 1], nullptr);
        HIP_OK(hipDeviceSynchronize());
        nn->have_map = true;
        return SG_OK;
    });
}

int nn_forward(sg_nn* nn, const double* X, int B, double* U, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(nn && X && U, "null argument");
        SG_REQUIRE(B >= 1 && B <= nn->max_batch, "batch %d outside [1,%d]", B, nn->max_batch);
        SG_REQUIRE(nn->have_map, "output map (env, oscale) not set");
        check_device(nn->device);
        hipStream_t s = as_stream(stream);
        nn_forward_core(nn, X, B, s);
        const int64_t npix = (int64_t)B * nn->H * nn->W;
        const int L = nn->nl;
        predict_kernel<<<blocks_for(npix * nn->co[L - 1]), kNT, 0, s>>>(
            npix, nn->H * nn->W, nn->co[L - 1], nn->cop[L - 1], nn->out.p, nn->env.p, nn->oscale.p, U);
        HIP_LAUNCH_OK();
        return SG_OK;
    });
}

int nn_loss_grad(sg_nn* nn, const double* X, const double* T, int B, double* loss, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(nn && X && T, "null argument");
        SG_REQUIRE(B >= 1 && B <= nn->max_batch, "batch %d outside [1,%d]", B, nn->max_batch);
        check_device(nn->device);
        const double l = nn_backward_core(nn, X, T, B, as_stream(stream));
        if (loss) *loss = l;
        return SG_OK;
    });
}

int nn_adam_step(sg_nn* nn, float lr, float beta1, float beta2, float eps, void* stream) {
    return guarded([&]() -> int {
        SG_REQUIRE(nn != nullptr, "nn is NULL");
        SG_REQUIRE(lr > 0.f && beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f &&
                       eps > 0.f, "bad Adam hyper-parameters");
        check_device(nn->device);
        hipStream_t s = as_stream(stream);
        nn->t += 1;
        const float c1 = 1.f - std::pow(beta1, (float)nn->t);
        const float c2 = 1.f - std::pow(beta2, (float)nn->t);
        adam_kernel<<<blocks_for(nn->nparam), kNT, 0, s>>>(nn->nparam, lr, beta1, beta2, eps, c1, c2,
                                                           nn->p.p, nn->g.p, nn->m.p, nn->v.p);
        HIP_LAUNCH_OK();
        pack_weights(nn, s);
        return SG_OK;
    });
}

void nn_destroy(sg_nn* nn) { delete nn; }

}  // extern "C"
