// unet.hip -- a small U-Net on the structured nodal grid, trained and applied
// with hand-written BF16 MFMA kernels (FP32 accumulation).  It serves as the
// preconditioner of flexible CG (fcg.hip).
//
// Network (base width c; NHWC BF16 activations; level l has (H>>l) x (W>>l)):
//   L0  conv3x3(8 -> c) ReLU          L1  conv3x3(c -> c) ReLU       = e0
//   pool; L2 conv(c -> 2c) ReLU;      L3  conv(2c -> 2c) ReLU        = e1
//   pool; L4 conv(2c -> 4c) ReLU;     L5  conv(4c -> 4c) ReLU        = e2
//   pool; L6 conv(4c -> 8c) ReLU;     L7  conv(8c -> 8c) ReLU        = m
//   L8  upconv2x2(8c -> 4c);  L9  conv([u2, e2] -> 4c) ReLU;  L10 conv(4c -> 4c) ReLU = d2
//   L11 upconv2x2(4c -> 2c);  L12 conv([u1, e1] -> 2c) ReLU;  L13 conv(2c -> 2c) ReLU = d1
//   L14 upconv2x2(2c -> c);   L15 conv([u0, e0] -> c) ReLU;   L16 conv(c -> c) ReLU   = d0
//   out conv1x1(c -> 1), FP32
// pool = 2x2 average; the input has 2 channels (scaled residual, constant
// channel) stored as 8 so that every MFMA fragment reads 8 channels.
//
// Every convolution is an implicit GEMM on v_mfma_f32_16x16x32_bf16: rows are
// pixels (16 per wave, 64 per workgroup), columns output channels, and the
// reduction runs over (tap, input channel) in blocks of 32.  Each lane loads 8
// consecutive channels of one pixel (16 bytes) and 8 reduction rows of the
// weight fragment, which is kept pre-packed in MFMA operand order.
// Backward-data is the same GEMM on the ReLU-masked output gradient with the
// transposed weights.  Weight gradients reduce over pixels in fixed slices
// whose FP32 partials are added in slice order, so a training step is bitwise
// reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "common.h"
#include "fem.h"
#include "kernels.h"
#include "unet.h"

namespace fem {

namespace {

typedef __bf16 bf16;
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));

constexpr int kPixTile = 64;   // pixels per GEMM workgroup (4 waves x 16)

// Bytes of a conv tile's staged input (TY + 2) x (TX + 2) pixels x Cin BF16,
// rounded to 16.
__host__ __device__ constexpr size_t conv_tile_bytes(int TY, int TX, int Cin) {
    return ((size_t)(TY + 2) * (TX + 2) * Cin * 2 + 15) & ~(size_t)15;
}
// Reduction blocks of weights per LDS stage of the tiled convolution (1 KiB
// per block and column tile): all KB in one stage when they take at most
// 16 KiB; otherwise two alternating stages of at most 16 KiB each within the
// 64 KiB budget left by the input tile.
__host__ __device__ constexpr int conv_kbc(int KB, int NT, size_t tile) {
    return KB * NT <= 16 ? KB
                         : ((int)((65536 - (tile < 65536 ? tile : 65536)) / (2 * 1024 * NT)) < 16 / NT
                                ? ((int)((65536 - (tile < 65536 ? tile : 65536)) / (2 * 1024 * NT)) > 0
                                       ? (int)((65536 - (tile < 65536 ? tile : 65536)) / (2 * 1024 * NT))
                                       : 1)
                                : (16 / NT > 0 ? 16 / NT : 1));
}
// LDS of the tiled convolution: input tile and one or two weight stages
__host__ __device__ constexpr size_t conv_lds_bytes(int TY, int TX, int Cin, int KB, int NT) {
    return conv_tile_bytes(TY, TX, Cin) +
           (size_t)(KB * NT <= 16 ? 1 : 2) * conv_kbc(KB, NT, conv_tile_bytes(TY, TX, Cin)) * NT * 1024;
}
constexpr int kWSlice = 4096;  // pixels per weight-gradient slice

__device__ __forceinline__ f4 mfma(bf8 a, bf8 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }

__device__ __forceinline__ bf8 zero8() {
    bf8 z;
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = (bf16)0.0f;
    return z;
}

__device__ __forceinline__ bf8 ld8(const bf16 *p) { return *reinterpret_cast<const bf8 *>(p); }

// ---------------------------------------------------------------------------
// A-operand sources: 8 consecutive reduction entries (k0 .. k0+7) of row m.
// ---------------------------------------------------------------------------

// conv3x3 forward: row m = pixel (b, y, x); k = tap * Cin + ci, tap = ky*3+kx;
// channels [0, C1) from src1, [C1, C1 + C2) from src2 (concatenation).
// Each source splits its row m once per lane (row()) and then loads the
// reduction entries of that row (load(row, k0)), so the pixel arithmetic is not
// repeated for every reduction block.
struct SrcConv {
    const bf16 *src1, *src2;
    int C1, C2, H, W;
    struct Row {
        int m, x, y;
    };
    __device__ __forceinline__ Row row(int m) const { return {m, m % W, (m / W) % H}; }
    __device__ __forceinline__ bf8 load(const Row &rw, int k0) const {
        const int Cin = C1 + C2;
        const int tap = k0 / Cin, ci = k0 - tap * Cin;
        if (tap >= 9) return zero8();
        const int m = rw.m, x = rw.x, y = rw.y;
        const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
        if (yy < 0 || yy >= H || xx < 0 || xx >= W) return zero8();
        const int64_t pix = (int64_t)m + (int64_t)(tap / 3 - 1) * W + (tap % 3 - 1);
        if (ci < C1) return ld8(src1 + pix * C1 + ci);
        return ld8(src2 + pix * C2 + (ci - C1));
    }
};

// conv3x3 backward-data: row m = input pixel q; k = tap * Cout + co, entry
// gz[q - d_tap][co] with gz = gy * (y > 0).
struct SrcConvBwd {
    const bf16 *gy, *y;
    int Cout, lcout, H, W;  // Cout = 2^lcout
    struct Row {
        int m, x, yq;
    };
    __device__ __forceinline__ Row row(int m) const { return {m, m % W, (m / W) % H}; }
    __device__ __forceinline__ bf8 load(const Row &rw, int k0) const {
        const int tap = k0 >> lcout, co = k0 & (Cout - 1);
        if (tap >= 9) return zero8();
        const int m = rw.m, x = rw.x, yq = rw.yq;
        // tap t of the packed (flipped) weights reads pixel (y + t/3 - 1, x + t%3 - 1),
        // the geometry of the forward convolution
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const int yy = yq + dy, xx = x + dx;
        if (yy < 0 || yy >= H || xx < 0 || xx >= W) return zero8();
        const int64_t off = ((int64_t)m + (int64_t)dy * W + dx) * Cout + co;
        bf8 g = ld8(gy + off);
        const bf8 v = ld8(y + off);
#pragma unroll
        for (int i = 0; i < 8; ++i) g[i] = ((float)v[i] > 0.0f) ? g[i] : (bf16)0.0f;
        return g;
    }
};

// rows of a [M][C] tensor (up-conv forward: m = low-resolution pixel)
struct SrcRows {
    const bf16 *src;
    int C;
    using Row = int;
    __device__ __forceinline__ Row row(int m) const { return m; }
    __device__ __forceinline__ bf8 load(int m, int k0) const {
        if (k0 >= C) return zero8();
        return ld8(src + (int64_t)m * C + k0);
    }
};

__device__ __forceinline__ int64_t fine_pixel(int m, int q, int H, int W) {
    // low pixel m = (b, y, x) of an H x W level -> fine pixel (b, 2y + q/2, 2x + q%2)
    const int x = m % W, t = m / W, y = t % H, b = t / H;
    return ((int64_t)b * 2 * H + 2 * y + (q >> 1)) * (2 * W) + 2 * x + (q & 1);
}

// up-conv backward-data: row m = low pixel; k = q * Cout + co, entry du[fine(m, q)][co]
struct SrcUpBwd {
    const bf16 *du;
    int Cout, H, W;  // low resolution
    using Row = int;
    __device__ __forceinline__ Row row(int m) const { return m; }
    __device__ __forceinline__ bf8 load(int m, int k0) const {
        const int q = k0 / Cout, co = k0 - q * Cout;
        if (q >= 4) return zero8();
        return ld8(du + fine_pixel(m, q, H, W) * Cout + co);
    }
};

// ---------------------------------------------------------------------------
// Epilogues: value v of row m, column n.
// ---------------------------------------------------------------------------
struct EpiConv {  // bias + ReLU -> bf16 [M][N]
    bf16 *out;
    const float *bias;
    int N;
    __device__ __forceinline__ void put(int m, int n, float v) const {
        v += bias[n];
        out[(int64_t)m * N + n] = (bf16)(v > 0.0f ? v : 0.0f);
    }
};

struct EpiGrad {  // gradient of a (possibly concatenated) input: columns [0,C1) -> g1, the rest -> g2
    bf16 *g1, *g2;
    int C1, C2;
    __device__ __forceinline__ void put(int m, int n, float v) const {
        if (n < C1)
            g1[(int64_t)m * C1 + n] = (bf16)v;
        else if (g2)
            g2[(int64_t)m * C2 + (n - C1)] = (bf16)v;
    }
};

struct EpiUp {  // up-conv forward: column n = q*Cout + co -> out[fine(m, q)][co] (+ bias)
    bf16 *out;
    const float *bias;
    int Cout, H, W;  // low resolution
    __device__ __forceinline__ void put(int m, int n, float v) const {
        const int q = n / Cout, co = n - q * Cout;
        out[fine_pixel(m, q, H, W) * Cout + co] = (bf16)(v + bias[co]);
    }
};

// Row GEMM D[M][16 NT] = A[M][32 KB] B[32 KB][16 NT]; Bp holds B in fragment
// order [KB][NT][64 lanes][8].  Each wave owns 16 rows and all columns.
template <class Src, class Epi, int NT>
__global__ __launch_bounds__(256) void k_gemm_rows(Src src, Epi epi, const bf16 *__restrict__ Bp, int M, int KB) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = blockIdx.x * kPixTile + wave * 16;
    if (m0 >= M) return;
    f4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    const int mr = m0 + (lane & 15);
    const bool row_ok = mr < M;
    const typename Src::Row rw = src.row(row_ok ? mr : m0);
    for (int kb = 0; kb < KB; ++kb) {
        const bf8 a = row_ok ? src.load(rw, kb * 32 + 8 * (lane >> 4)) : zero8();
        const bf16 *bk = Bp + ((int64_t)kb * NT * 64 + lane) * 8;
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mfma(a, ld8(bk + (int64_t)t * 64 * 8), acc[t]);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int m = m0 + 4 * (lane >> 4) + i;
            if (m < M) epi.put(m, t * 16 + (lane & 15), acc[t][i]);
        }
}

// LDS-tiled 3x3 convolution forward (+ bias, ReLU).  A workgroup of 4 waves
// owns a TY x TX pixel tile of one image: the tile's input with a one-pixel
// halo ([C1 channels of src1 | CIN - C1 of src2]) is staged in LDS once, so
// every input value is read once per tile instead of once per tap; the packed
// weight fragments are staged in blocks of KBC reduction blocks (all of them
// when they fit in 16 KiB, else two alternating stages, the next one loaded
// while the current one is used), shared by the 4 waves.  Wave w computes tile
// pixels [64 MT/4 * w ...) as MT tiles of 16 pixels against all NT tiles of
// 16 output channels.  The product is taken transposed, D^T = W^T A^T: the
// weight fragment is the MFMA's first operand (rows = output channels) and the
// pixels its second, so that each lane ends with four consecutive output
// channels of one pixel and stores them as one 8-byte word, sixteen lanes
// covering 16 consecutive pixels of an NHWC row.  CIN is a template constant,
// so the (tap, channel) of every reduction block is a shift and a mask of
// compile-time values and the reduction loop is unrolled.  Pixels outside the
// image are computed on zero input and not stored; reduction entries past the
// 9 taps (padding of the last block) have zero weights and read the last
// tap's finite inputs.
template <int TY, int TX, int NTA, int CIN, int NS = 1, bool BWD = false, bool POOL = false>
__global__ __launch_bounds__(256) void k_conv3x3(const bf16 *__restrict__ src1, const bf16 *__restrict__ src2, int C1,
                                                 int H, int W, int tiles_x, int tiles_y, const bf16 *__restrict__ Bp,
                                                 const float *__restrict__ bias, bf16 *__restrict__ out,
                                                 bf16 *__restrict__ out2, int C1o) {
    // NS workgroups share a pixel tile, each computing NT = NTA / NS of its
    // NTA column tiles (output channels [split * 16 NT, (split + 1) * 16 NT))
    constexpr int NT = NTA / NS;
    static_assert(NT * NS == NTA && NT >= 1, "column split");
    constexpr int MT = TY * TX / 64;
    constexpr int HX = TX + 2, HY = TY + 2;
    constexpr int KB = (9 * CIN + 31) / 32;
    constexpr int KBC = conv_kbc(KB, NT, conv_tile_bytes(TY, TX, CIN));
    constexpr int NBLK = (KB + KBC - 1) / KBC;  // weight stages
    constexpr int FR = (KBC * NT * 64 + 255) / 256;  // weight fragments per thread and stage
    constexpr int CU8 = CIN / 8;
    constexpr int N = NTA * 16;  // output channels (the NHWC pitch)
    static_assert(CIN >= 8 && (CIN & (CIN - 1)) == 0, "CIN must be a power of two >= 8");
    static_assert(TX % 16 == 0 && (TY * TX) % 64 == 0, "tile shape");
    extern __shared__ __align__(16) unsigned char smem[];
    bf16 *tin = reinterpret_cast<bf16 *>(smem);  // [HY * HX][CIN]
    bf8 *tb0 = reinterpret_cast<bf8 *>(smem + conv_tile_bytes(TY, TX, CIN));  // [KBC][NT][64], two when NBLK > 1
    bf8 *tb1 = tb0 + KBC * NT * 64;
    const int C2 = CIN - C1;
    const int split = NS > 1 ? (int)(blockIdx.x % NS) : 0;
    const int tile = NS > 1 ? (int)(blockIdx.x / NS) : (int)blockIdx.x;
    const int c0 = split * NT * 16;  // first output channel of this workgroup
    const int tx = tile % tiles_x, t2 = tile / tiles_x, ty = t2 % tiles_y, b = t2 / tiles_y;
    const int y0 = ty * TY, x0 = tx * TX;
    const int64_t img = (int64_t)b * H * W;
    for (int u = threadIdx.x; u < HY * HX * CU8; u += 256) {
        const int cu = u % CU8, pp = u / CU8;
        const int yy = y0 + pp / HX - 1, xx = x0 + pp % HX - 1;
        bf8 v = zero8();
        if ((unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)W) {
            const int64_t pix = img + (int64_t)yy * W + xx;
            const int ci = cu * 8;
            if constexpr (BWD) {
                // the output gradient where the layer's ReLU passed (src2: its output)
                v = ld8(src1 + pix * CIN + ci);
                const bf8 a = ld8(src2 + pix * CIN + ci);
#pragma unroll
                for (int i = 0; i < 8; ++i) v[i] = ((float)a[i] > 0.0f) ? v[i] : (bf16)0.0f;
            } else {
                v = ci < C1 ? ld8(src1 + pix * C1 + ci) : ld8(src2 + pix * C2 + (ci - C1));
            }
        }
        *reinterpret_cast<bf8 *>(tin + pp * CIN + cu * 8) = v;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4;
    int hoff[MT];  // LDS element offset of this lane's pixel in row tile mt
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int p = (wave * MT + mt) * 16 + (lane & 15);
        hoff[mt] = ((p / TX) * HX + p % TX) * CIN;
    }
    f4 acc[MT][NT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[mt][t] = f4{0.f, 0.f, 0.f, 0.f};
    const bf8 *wsrc = reinterpret_cast<const bf8 *>(Bp);
    // stage element u = (kb - kc) NT 64 + t 64 + lane of reduction block kb
    // comes from packed fragment (kb NTA + split NT + t) 64 + lane
    auto wsel = [&](int kc, int u) -> size_t {
        if constexpr (NS == 1) {
            return (size_t)kc * NT * 64 + u;
        } else {
            const int kr = u / (NT * 64), rem = u - kr * (NT * 64);
            return ((size_t)(kc + kr) * NTA + split * NT) * 64 + rem;
        }
    };
    {
        constexpr int n0 = (KBC < KB ? KBC : KB) * NT * 64;
        for (int u = threadIdx.x; u < n0; u += 256) tb0[u] = wsrc[wsel(0, u)];
    }
    __syncthreads();  // input tile and the first weight stage
    // stage j + 1 is loaded into registers while stage j is computed, then
    // stored into the other buffer behind one barrier
#pragma unroll
    for (int j = 0; j < NBLK; ++j) {
        const int kc = j * KBC;
        bf8 nxt[FR];
        const int n1 = (j + 1 < NBLK) ? ((KB - kc - KBC < KBC ? KB - kc - KBC : KBC) * NT * 64) : 0;
        if (j + 1 < NBLK) {
#pragma unroll
            for (int f = 0; f < FR; ++f) {
                const int u = threadIdx.x + f * 256;
                if (u < n1) nxt[f] = wsrc[wsel(kc + KBC, u)];
            }
        }
        const bf8 *tb = (j & 1) ? tb1 : tb0;
#pragma unroll
        for (int kl = 0; kl < KBC; ++kl) {
            if (kc + kl < KB) {
                // this lane's reduction entries (kc + kl) * 32 + 8 g .. + 7: one tap, 8 channels
                const int k0 = (kc + kl) * 32 + 8 * g;
                int tap = k0 / CIN;
                tap = tap < 9 ? tap : 8;
                const int toff = ((tap / 3) * HX + tap % 3) * CIN + (k0 % CIN);
                bf8 a[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) a[mt] = *reinterpret_cast<const bf8 *>(tin + hoff[mt] + toff);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const bf8 wv = tb[(kl * NT + t) * 64 + lane];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) acc[mt][t] = mfma(wv, a[mt], acc[mt][t]);
                }
            }
        }
        if (j + 1 < NBLK) {
            bf8 *tn = (j & 1) ? tb0 : tb1;
#pragma unroll
            for (int f = 0; f < FR; ++f) {
                const int u = threadIdx.x + f * 256;
                if (u < n1) tn[u] = nxt[f];
            }
            __syncthreads();  // stage j + 1 stored; every wave is done with stage j - 1's buffer
        }
    }
    // lane: pixel (lane & 15) of row tile mt, output channels t * 16 + 4 g .. + 3
    const bool full = y0 + TY <= H && x0 + TX <= W;  // no pixel of the tile outside the image
    if constexpr (BWD) {
        // input gradient, no bias or ReLU: channels [0, C1o) -> out (pitch C1o),
        // the rest -> out2 (pitch N - C1o); C1o is a multiple of 16, so each
        // column tile lies in one of them
        const int C2o = N - C1o;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int p = (wave * MT + mt) * 16 + (lane & 15);
            const int py = p / TX, px = p % TX;
            if (full || (y0 + py < H && x0 + px < W)) {
                const int64_t pix = img + (int64_t)(y0 + py) * W + (x0 + px);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int c = c0 + t * 16 + 4 * g;
                    bf4 r;
#pragma unroll
                    for (int i = 0; i < 4; ++i) r[i] = (bf16)acc[mt][t][i];
                    if (c < C1o) *reinterpret_cast<bf4 *>(out + pix * C1o + c) = r;
                    else if (out2) *reinterpret_cast<bf4 *>(out2 + pix * C2o + (c - C1o)) = r;
                }
            }
        }
    } else {
        float bv[NT][4];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) bv[t][i] = bias[c0 + t * 16 + 4 * g + i];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int p = (wave * MT + mt) * 16 + (lane & 15);
            const int py = p / TX, px = p % TX;
            if (full || (y0 + py < H && x0 + px < W)) {
                bf16 *o = out + (img + (int64_t)(y0 + py) * W + (x0 + px)) * N + c0 + 4 * g;
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    bf4 r;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float v = acc[mt][t][i] + bv[t][i];
                        r[i] = (bf16)(v > 0.0f ? v : 0.0f);
                    }
                    *reinterpret_cast<bf4 *>(o + t * 16) = r;
                }
            }
        }
        if constexpr (POOL) {
            // 2 x 2 average pooling of the tile into out2 ((H/2) x (W/2), N
            // channels), from the same BF16 values and with the expression of
            // k_pool_fwd: the tile's outputs go to LDS once every wave is done
            // with the input tile
            static_assert(NS == 1 && TY % 2 == 0 && TX % 2 == 0, "pooling needs the whole tile");
            __syncthreads();
            bf16 *tout = tin;  // [TY * TX][N]
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const int p = (wave * MT + mt) * 16 + (lane & 15);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    bf4 r;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const float v = acc[mt][t][i] + bv[t][i];
                        r[i] = (bf16)(v > 0.0f ? v : 0.0f);
                    }
                    *reinterpret_cast<bf4 *>(tout + p * N + t * 16 + 4 * g) = r;
                }
            }
            __syncthreads();
            const int H2 = H / 2, W2 = W / 2;
            constexpr int c8 = N / 8;
            for (int i = threadIdx.x; i < (TY / 2) * (TX / 2) * c8; i += 256) {
                const int cg = i % c8, pp = i / c8, px = pp % (TX / 2), py = pp / (TX / 2);
                const int Y = y0 / 2 + py, X = x0 / 2 + px;
                if (Y >= H2 || X >= W2) continue;
                const bf16 *q = tout + ((2 * py) * TX + 2 * px) * N + cg * 8;
                const bf8 a = *reinterpret_cast<const bf8 *>(q), bb = *reinterpret_cast<const bf8 *>(q + N),
                          c = *reinterpret_cast<const bf8 *>(q + TX * N),
                          d = *reinterpret_cast<const bf8 *>(q + TX * N + N);
                bf8 r;
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    r[k] = (bf16)(0.25f * (((float)a[k] + (float)bb[k]) + ((float)c[k] + (float)d[k])));
                *reinterpret_cast<bf8 *>(out2 + (((int64_t)b * H2 + Y) * W2 + X) * N + cg * 8) = r;
            }
        }
    }
}

// 2 x 2 stride-2 transposed convolution forward (+ bias): rows are the M
// low-resolution pixels, columns n = q * Cout + co with q = 2 a + c the fine
// position (2y + a, 2x + c), reduction over the Cin input channels.  As in
// k_conv3x3 the product is taken transposed (weight fragment first), so each
// lane ends with four consecutive output channels of one (pixel, q) and stores
// them as one 8-byte word; the lane's low pixel is decomposed into
// (image, y, x) once.  Cout (a multiple of 16, so the 16 columns of a tile
// share q) and the level's H and W are powers of two: the splits are shifts.
template <int NT>
__global__ __launch_bounds__(256) void k_upconv(const bf16 *__restrict__ in, int Cin, int lcout, int lh, int lw, int M,
                                                const bf16 *__restrict__ Bp, int KB, const float *__restrict__ bias,
                                                bf16 *__restrict__ out) {
    const int Cout = 1 << lcout, H = 1 << lh, W = 1 << lw;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4;
    const int m0 = blockIdx.x * kPixTile + wave * 16;
    if (m0 >= M) return;  // uniform across the wave
    const int mr = m0 + (lane & 15);
    const bool row_ok = mr < M;
    f4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    for (int kb = 0; kb < KB; ++kb) {
        const int k0 = kb * 32 + 8 * g;
        const bf8 a = (row_ok && k0 < Cin) ? ld8(in + (int64_t)mr * Cin + k0) : zero8();
        const bf8 *bk = reinterpret_cast<const bf8 *>(Bp) + (int64_t)kb * NT * 64 + lane;
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mfma(bk[t * 64], a, acc[t]);
    }
    if (!row_ok) return;
    const int x = mr & (W - 1), yb = mr >> lw, y = yb & (H - 1), b = yb >> lh;
    const int64_t W2 = 2 * (int64_t)W;
    const int64_t base = ((int64_t)b * 2 * H + 2 * y) * W2 + 2 * x;  // fine pixel of q = 0
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int n0 = t * 16 + 4 * g;
        const int q = n0 >> lcout, co = n0 & (Cout - 1);
        const int64_t fine = base + (q >> 1) * W2 + (q & 1);
        bf4 r;
#pragma unroll
        for (int i = 0; i < 4; ++i) r[i] = (bf16)(acc[t][i] + bias[co + i]);
        *reinterpret_cast<bf4 *>(out + fine * Cout + co) = r;
    }
}

// ---------------------------------------------------------------------------
// Weight gradients: dW[r][n] = sum_pixels A[pixel][r] G[pixel][n]; the rows r
// are those of the im2col operand plus a last bias row of ones.  Workgroup
// (i, s) computes rows [64 i, 64 i + 64) over the pixel slice s into
// partial[s][R1][N]; the slices are added in order afterwards.
// ---------------------------------------------------------------------------
// a8 / g8 return the operand for the 8 consecutive pixels p .. p + 7 of one
// lane (0 from p1 on).  When the 8 pixels lie in one image row (W a multiple
// of 8; p is then a multiple of 8) the pixel's row and column are computed
// once, not per entry; otherwise entry by entry.  Same values either way.
struct WSrcConv {  // conv3x3: r = tap * Cin + ci; r == R is the bias row
    const bf16 *src1, *src2;
    int C1, C2, H, W, R;
    __device__ __forceinline__ float a(int64_t pix, int r) const {
        if (r == R) return 1.0f;
        const int Cin = C1 + C2;
        const int tap = r / Cin, ci = r - tap * Cin;
        const int x = (int)(pix % W);
        const int y = (int)((pix / W) % H);
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        if (y + dy < 0 || y + dy >= H || x + dx < 0 || x + dx >= W) return 0.0f;
        const int64_t q = pix + (int64_t)dy * W + dx;
        return ci < C1 ? (float)src1[q * C1 + ci] : (float)src2[q * C2 + (ci - C1)];
    }
    __device__ __forceinline__ bf8 a8(int64_t p, int r, int64_t p1) const {
        bf8 v;
        if (r == R || p + 8 > p1 || (W & 7)) {
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = (bf16)(p + i < p1 ? a(p + i, r) : 0.0f);
            return v;
        }
        const int Cin = C1 + C2;
        const int tap = r / Cin, ci = r - tap * Cin;
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const int64_t row = p / W;
        const int x0 = (int)(p - row * W);
        const int y = (int)(row % H);
        if (y + dy < 0 || y + dy >= H) return zero8();
        const bool first = ci < C1;
        const int C = first ? C1 : C2;
        const bf16 *base = (first ? src1 + ci : src2 + (ci - C1)) + (p + (int64_t)dy * W + dx) * C;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int xx = x0 + i + dx;
            v[i] = (xx >= 0 && xx < W) ? base[(int64_t)i * C] : (bf16)0.0f;
        }
        return v;
    }
};
struct WGradConv {  // gy * (y > 0)
    const bf16 *gy, *y;
    int N;
    using Prep = int;
    __device__ __forceinline__ Prep prep(int64_t) const { return 0; }
    __device__ __forceinline__ bf8 g8(Prep, int64_t p, int n, int64_t p1) const { return g8(p, n, p1); }
    __device__ __forceinline__ float g(int64_t pix, int n) const {
        const int64_t o = pix * N + n;
        return (float)y[o] > 0.0f ? (float)gy[o] : 0.0f;
    }
    __device__ __forceinline__ bf8 g8(int64_t p, int n, int64_t p1) const {
        bf8 v;
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = (bf16)(p + i < p1 ? g(p + i, n) : 0.0f);
        return v;
    }
};
struct WSrcUp {  // up-conv: r = ci; r == C is the bias row
    const bf16 *src;
    int C;
    __device__ __forceinline__ float a(int64_t pix, int r) const { return r == C ? 1.0f : (float)src[pix * C + r]; }
    __device__ __forceinline__ bf8 a8(int64_t p, int r, int64_t p1) const {
        bf8 v;
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = (bf16)(p + i < p1 ? a(p + i, r) : 0.0f);
        return v;
    }
};
struct WGradUp {  // column n = q * Cout + co: du at the fine position q of low pixel pix
    const bf16 *du;
    int Cout, H, W;
    // fine pixel of q = 0 for the lane's 8 low pixels p .. p + 7 (one image row
    // when W is a multiple of 8; -1: take the entry-by-entry path), computed
    // once per reduction step instead of once per column tile
    using Prep = int64_t;
    __device__ __forceinline__ Prep prep(int64_t p) const {
        if (W & 7) return -1;
        const int x = (int)(p % W), yb = (int)(p / W), y = yb % H, b = yb / H;
        return ((int64_t)b * 2 * H + 2 * y) * (2 * (int64_t)W) + 2 * x;
    }
    __device__ __forceinline__ bf8 g8(Prep f0, int64_t p, int n, int64_t p1) const {
        if (f0 < 0 || p + 8 > p1) return g8(p, n, p1);
        const int q = n / Cout, co = n - q * Cout;
        const bf16 *base = du + (f0 + (q >> 1) * 2 * (int64_t)W + (q & 1)) * Cout + co;
        bf8 v;
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = base[(int64_t)2 * i * Cout];
        return v;
    }
    __device__ __forceinline__ float g(int64_t pix, int n) const {
        const int q = n / Cout, co = n - q * Cout;
        return (float)du[fine_pixel((int)pix, q, H, W) * Cout + co];
    }
    __device__ __forceinline__ bf8 g8(int64_t p, int n, int64_t p1) const {
        bf8 v;
        if (p + 8 > p1 || (W & 7)) {
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = (bf16)(p + i < p1 ? g(p + i, n) : 0.0f);
            return v;
        }
        // low pixels p .. p+7 share a row: their fine pixels are 2 apart
        const int q = n / Cout, co = n - q * Cout;
        const bf16 *base = du + fine_pixel((int)p, q, H, W) * Cout + co;
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = base[(int64_t)2 * i * Cout];
        return v;
    }
};

// XCD-aware decomposition of a weight-gradient grid into (row block, slice).
// Workgroups are dealt to the kXcds XCDs in turn, so block b runs on XCD
// b % kXcds; the row blocks of one slice get ids that share b % kXcds and
// follow each other on that XCD (k = b / kXcds runs over the row blocks
// first), so that the slice's output-gradient and input tiles, which every
// row block reads, come through that XCD's L2 instead of from HBM once per
// row block.  The grid has nrb * ceil(splits / kXcds) * kXcds blocks; those
// past the last slice return at once.
constexpr int kXcds = 8;
struct WTile {
    int rb, s;
};
__device__ __forceinline__ WTile wgrad_tile(int nrb) {
    const int b = blockIdx.x, x = b % kXcds, k = b / kXcds;
    return {k % nrb, (k / nrb) * kXcds + x};
}
inline unsigned wgrad_grid(int nrb, int64_t splits) {
    return (unsigned)((int64_t)nrb * ((splits + kXcds - 1) / kXcds) * kXcds);
}

template <class WS, class WG, int NT>
__global__ __launch_bounds__(256) void k_gemm_wgrad(WS ws, WG wg, int R1, int N, int64_t P, int64_t slice,
                                                    float *__restrict__ partial) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const WTile tl = wgrad_tile((R1 + 63) / 64);
    if ((int64_t)tl.s * slice >= P) return;
    const int r0 = tl.rb * 64 + wave * 16;
    if (r0 >= R1) return;
    const int s = tl.s;
    const int64_t p0 = (int64_t)s * slice, p1 = std::min<int64_t>(P, p0 + slice);
    f4 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    const int r = r0 + (lane & 15);
    for (int64_t pb = p0; pb < p1; pb += 32) {
        const int64_t pl = pb + 8 * (lane >> 4);  // this lane's 8 pixels
        const bf8 a = r < R1 ? ws.a8(pl, r, p1) : zero8();
        const typename WG::Prep pr = wg.prep(pl);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int n = t * 16 + (lane & 15);
            const bf8 bv = n < N ? wg.g8(pr, pl, n, p1) : zero8();
            acc[t] = mfma(a, bv, acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rr = r0 + 4 * (lane >> 4) + i, n = t * 16 + (lane & 15);
            if (rr < R1 && n < N) partial[((int64_t)s * R1 + rr) * N + n] = acc[t][i];
        }
}

// Conv3x3 weight gradients with both operands staged through LDS.  For each
// chunk of kWChunk pixels of its slice, workgroup (i, s) loads the 64 im2col
// rows [64 i, 64 i + 64) and the masked output gradient gy * (y > 0) with
// 16-byte loads (8 consecutive channels of one pixel: a row group shares its
// tap when the channel counts are multiples of 8) and stores them transposed,
// [row][pixel], so that each lane reads its 8 consecutive pixels of a row with
// one 16-byte LDS read.  The MFMA operands, their order and the partials are
// exactly those of k_gemm_wgrad<WSrcConv, WGradConv>.
constexpr int kWChunk = 128;
constexpr int kWPitch = kWChunk + 8;  // LDS row pitch in bf16 (272 bytes: 16-byte aligned rows)

// RT row tiles of 16 per wave: a workgroup covers 64 RT im2col rows, so the
// masked output gradient staged per chunk serves RT times as many MFMAs.
template <int NT, int RT = 1>
__global__ __launch_bounds__(256) void k_wgrad_conv(WSrcConv ws, WGradConv wg, int R1, int N, int64_t P, int64_t slice,
                                                    float *__restrict__ partial) {
    __shared__ __align__(16) bf16 sa[64 * RT * kWPitch];
    __shared__ __align__(16) bf16 sg[NT * 16 * kWPitch];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const WTile tl = wgrad_tile((R1 + 64 * RT - 1) / (64 * RT));
    if ((int64_t)tl.s * slice >= P) return;  // uniform: before any barrier
    const int rb = tl.rb * 64 * RT;
    const int r0 = rb + wave * RT * 16;  // first row of this wave's RT row tiles
    const int s = tl.s;
    const int64_t p0 = (int64_t)s * slice, p1 = std::min<int64_t>(P, p0 + slice);
    const int Cin = ws.C1 + ws.C2, H = ws.H, W = ws.W;
    f4 acc[RT][NT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[rt][t] = f4{0.f, 0.f, 0.f, 0.f};
    // A items (pixel pl, group rg of 8 rows): each thread keeps one pixel
    // column and 4 RT row groups; their (tap, channel) splits do not depend on
    // the chunk and are taken once
    constexpr int kRG = kWChunk * 8 * RT / 256;
    static_assert(kWChunk * 8 % 256 == 0 && 256 % kWChunk == 0, "A items per thread");
    const int pl = threadIdx.x % kWChunk;
    int rdy[kRG], rdx[kRG], rci[kRG], rkind[kRG];  // kind: 0 zero row, 1 bias row, 2 data row
#pragma unroll
    for (int j = 0; j < kRG; ++j) {
        const int rg = threadIdx.x / kWChunk + j * (256 / kWChunk);
        const int r = rb + 8 * rg;
        rkind[j] = r == ws.R ? 1 : (r < ws.R ? 2 : 0);
        const int tap = r < ws.R ? r / Cin : 0;
        rci[j] = r < ws.R ? r - tap * Cin : 0;
        rdy[j] = tap / 3 - 1;
        rdx[j] = tap % 3 - 1;
    }
    for (int64_t cb = p0; cb < p1; cb += kWChunk) {
        __syncthreads();  // the previous chunk's operands are consumed
        // the chunk's pixels cb .. cb + kWChunk - 1: image row and column of
        // the first one, once per chunk (uniform); they lie in one image row
        // when W is a multiple of the chunk length
        const int64_t row0 = cb / W;
        const int xc = (int)(cb - row0 * W), yc = (int)(row0 % H);
        const bool one_row = W % kWChunk == 0;
        const int64_t p = cb + pl;
        int x = xc + pl, y = yc;
        if (!one_row) {
            const int64_t row = p / W;
            x = (int)(p - row * W);
            y = (int)(row % H);
        }
#pragma unroll
        for (int j = 0; j < kRG; ++j) {
            const int rg = threadIdx.x / kWChunk + j * (256 / kWChunk);
            bf8 v = zero8();
            if (p < p1) {
                if (rkind[j] == 1) {
                    v[0] = (bf16)1.0f;  // bias row; rows R+1.. are beyond R1
                } else if (rkind[j] == 2) {
                    const int dy = rdy[j], dx = rdx[j], ci = rci[j];
                    if (y + dy >= 0 && y + dy < H && x + dx >= 0 && x + dx < W) {
                        const int64_t q = p + (int64_t)dy * W + dx;
                        v = ci < ws.C1 ? ld8(ws.src1 + q * ws.C1 + ci) : ld8(ws.src2 + q * ws.C2 + (ci - ws.C1));
                    }
                }
            }
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) sa[(8 * rg + jj) * kWPitch + pl] = v[jj];
        }
        // G: items (pixel, group of 8 output channels)
        for (int it = threadIdx.x; it < kWChunk * 2 * NT; it += 256) {
            const int pl = it % kWChunk, ng = it / kWChunk;
            const int64_t p = cb + pl;
            bf8 v = zero8();
            if (p < p1) {
                const bf8 g = ld8(wg.gy + p * N + 8 * ng), yv = ld8(wg.y + p * N + 8 * ng);
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = (float)yv[j] > 0.0f ? g[j] : (bf16)0.0f;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) sg[(8 * ng + j) * kWPitch + pl] = v[j];
        }
        __syncthreads();
        if (r0 < R1) {
            const int nks = (int)((std::min<int64_t>(p1 - cb, kWChunk) + 31) / 32);  // steps that start before p1
            for (int ks = 0; ks < nks; ++ks) {
                const int col = ks * 32 + 8 * (lane >> 4);
                bf8 bv[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    bv[t] = *reinterpret_cast<const bf8 *>(sg + (t * 16 + (lane & 15)) * kWPitch + col);
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    if (r0 + rt * 16 >= R1) break;  // uniform across the wave
                    const bf8 a =
                        *reinterpret_cast<const bf8 *>(sa + ((wave * RT + rt) * 16 + (lane & 15)) * kWPitch + col);
#pragma unroll
                    for (int t = 0; t < NT; ++t) acc[rt][t] = mfma(a, bv[t], acc[rt][t]);
                }
            }
        }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        if (r0 + rt * 16 >= R1) break;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int rr = r0 + rt * 16 + 4 * (lane >> 4) + i, n = t * 16 + (lane & 15);
                if (rr < R1 && n < N) partial[((int64_t)s * R1 + rr) * N + n] = acc[rt][t][i];
            }
    }
}

// sum_s x[s * stride], s = 0 .. splits-1 in order; kSumAhead loads are issued
// before they are added, so the ordered sum is not a chain of round trips
constexpr int kSumAhead = 32;
__device__ __forceinline__ float ordered_sum(const float *__restrict__ x, int splits, int64_t stride) {
    float v = 0.f;
    int s = 0;
    for (; s + kSumAhead <= splits; s += kSumAhead) {
        float t[kSumAhead];
#pragma unroll
        for (int j = 0; j < kSumAhead; ++j) t[j] = x[(int64_t)(s + j) * stride];
#pragma unroll
        for (int j = 0; j < kSumAhead; ++j) v += t[j];
    }
    for (; s < splits; ++s) v += x[(int64_t)s * stride];
    return v;
}

// Split sums with eight lanes per output: lane j adds, in order, the splits
// of its contiguous eighth of [0, splits), and the eight sums are combined by
// a fixed xor butterfly (commutative additions, so every lane of the group
// ends with the same value): the order is fixed for a given split count.
// Launch with kSumLanes threads per output (blockDim a multiple of 8).
constexpr int kSumLanes = 8;
__device__ __forceinline__ float lane_group_sum(float v) {
    v += __shfl_xor(v, 4, kSumLanes);
    v += __shfl_xor(v, 2, kSumLanes);
    v += __shfl_xor(v, 1, kSumLanes);
    return v;
}

// out[i] = sum_s partial[s][i]
__global__ void k_sum_splits(const float *__restrict__ partial, int splits, int64_t n, float *__restrict__ out) {
    const int j = threadIdx.x % kSumLanes;
    const int chunk = (splits + kSumLanes - 1) / kSumLanes;
    const int s0 = std::min(splits, j * chunk), s1 = std::min(splits, s0 + chunk);
    // the eight lanes of a group share i, so they run the same loop trips
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kSumLanes; i < n;
         i += (int64_t)gridDim.x * blockDim.x / kSumLanes) {
        const float v = lane_group_sum(ordered_sum(partial + (int64_t)s0 * n + i, s1 - s0, n));
        if (j == 0) out[i] = v;
    }
}

// up-conv: rows [0, Cin) of partial[s][Cin+1][4 Cout] are the weights; the
// bias row is summed over the 4 positions into out[Cin*4Cout + co]
// The same for the up-convolutions (the bias entries: the lane's splits for
// each of the four positions q in turn).
__global__ void k_sum_splits_up(const float *__restrict__ partial, int splits, int Cin, int Cout,
                                float *__restrict__ out) {
    const int64_t nw = (int64_t)Cin * 4 * Cout, n = nw + Cout, per = nw + 4 * Cout;
    const int j = threadIdx.x % kSumLanes;
    const int chunk = (splits + kSumLanes - 1) / kSumLanes;
    const int s0 = std::min(splits, j * chunk), s1 = std::min(splits, s0 + chunk);
    // every lane of a group runs the same number of loop trips (n is the same
    // for all of them), so the shuffles see all eight lanes
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kSumLanes; i < n;
         i += (int64_t)gridDim.x * blockDim.x / kSumLanes) {
        float v = 0.f;
        if (i < nw) {
            v = ordered_sum(partial + (int64_t)s0 * per + i, s1 - s0, per);
        } else {
            const int co = (int)(i - nw);
            for (int q = 0; q < 4; ++q) v += ordered_sum(partial + (int64_t)s0 * per + nw + q * Cout + co, s1 - s0, per);
        }
        v = lane_group_sum(v);
        if (j == 0) out[i] = v;
    }
}

// ---------------------------------------------------------------------------
// Elementwise and small kernels
// ---------------------------------------------------------------------------
// 2x2 average pooling, in [B][H][W][C] -> out [B][H/2][W/2][C]: one thread per
// 8 channels of an output pixel (16-byte loads and store; C a multiple of 8)
__global__ void k_pool_fwd(const bf16 *__restrict__ in, bf16 *__restrict__ out, int B, int H, int W, int C) {
    const int c8 = C / 8, W2 = W / 2, H2 = H / 2;
    const int64_t n = (int64_t)B * H2 * W2 * c8;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pix = i / c8;
        const int cg = (int)(i - pix * c8);
        const int x = (int)(pix % W2);
        const int64_t t = pix / W2;
        const int y = (int)(t % H2);
        const int64_t b = t / H2;
        const bf16 *p = in + ((b * H + 2 * y) * W + 2 * x) * C + cg * 8;
        const bf8 a = ld8(p), bb = ld8(p + C), c = ld8(p + (int64_t)W * C), d = ld8(p + (int64_t)W * C + C);
        bf8 r;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            r[k] = (bf16)(0.25f * (((float)a[k] + (float)bb[k]) + ((float)c[k] + (float)d[k])));
        *reinterpret_cast<bf8 *>(out + pix * C + cg * 8) = r;
    }
}

// gin (fine) += gout (coarse) / 4: one thread per 8 channels of a fine pixel
__global__ void k_pool_bwd(const bf16 *__restrict__ gout, bf16 *__restrict__ gin, int B, int H, int W, int C) {
    const int c8 = C / 8;
    const int64_t n = (int64_t)B * H * W * c8;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t pix = i / c8;
        const int cg = (int)(i - pix * c8);
        const int x = (int)(pix % W);
        const int64_t t = pix / W;
        const int y = (int)(t % H);
        const int64_t b = t / H;
        const bf8 g = ld8(gout + ((b * (H / 2) + y / 2) * (W / 2) + x / 2) * C + cg * 8);
        bf16 *q = gin + pix * C + cg * 8;
        bf8 v = ld8(q);
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = (bf16)((float)v[k] + 0.25f * (float)g[k]);
        *reinterpret_cast<bf8 *>(q) = v;
    }
}

// [P][2] fp32 -> [P][8] bf16 (channels 2..7 zero)
__global__ void k_make_input(const float *__restrict__ in2, bf16 *__restrict__ x8, int64_t P) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        bf8 v = zero8();
        v[0] = (bf16)in2[2 * p];
        v[1] = (bf16)in2[2 * p + 1];
        *reinterpret_cast<bf8 *>(x8 + p * 8) = v;
    }
}

// out[p] = b + sum_c d0[p][c] w[c]
__global__ void k_out_fwd(const bf16 *__restrict__ d0, const float *__restrict__ w, const float *__restrict__ bias,
                          int C, int64_t P, float *__restrict__ out) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        float s = bias[0];
        for (int c = 0; c < C; c += 8) {  // C is a multiple of 8: 16-byte loads
            const bf8 v = ld8(d0 + p * C + c);
#pragma unroll
            for (int i = 0; i < 8; ++i) s += (float)v[i] * w[c + i];
        }
        out[p] = s;
    }
}

// The 1x1 output layer and PASSES output smoothing passes in one launch: a
// workgroup owns a kHeadY x kHeadX tile of one image, evaluates the layer on
// the tile and a halo of PASSES pixels into LDS, runs the passes there (each
// on a region one pixel narrower per side) and stores the tile.  Every value
// is formed by the same expressions in the same order as in k_out_fwd
// followed by PASSES launches of k_binom, which it replaces.
constexpr int kHeadY = 16, kHeadX = 64;
template <int PASSES>
__global__ __launch_bounds__(256) void k_out_head(const bf16 *__restrict__ d0, const float *__restrict__ w,
                                                  const float *__restrict__ bias, int C, int H, int W, int tiles_x,
                                                  int tiles_y, float *__restrict__ out) {
    constexpr int RY = kHeadY + 2 * PASSES, RX = kHeadX + 2 * PASSES;
    __shared__ float buf[2][RY * RX];
    const int tile = blockIdx.x;
    const int tx = tile % tiles_x, t2 = tile / tiles_x, ty = t2 % tiles_y, b = t2 / tiles_y;
    const int gy0 = ty * kHeadY - PASSES, gx0 = tx * kHeadX - PASSES;  // image position of region pixel (0, 0)
    const int64_t img = (int64_t)b * H * W;
    for (int i = threadIdx.x; i < RY * RX; i += 256) {
        const int gy = gy0 + i / RX, gx = gx0 + i % RX;
        float s = 0.f;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) {
            const int64_t p = img + (int64_t)gy * W + gx;
            s = bias[0];
            for (int c = 0; c < C; c += 8) {
                const bf8 v = ld8(d0 + p * C + c);
#pragma unroll
                for (int j = 0; j < 8; ++j) s += (float)v[j] * w[c + j];
            }
        }
        buf[0][i] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PASSES; ++k) {
        const float *src = buf[k & 1];
        float *dst = buf[(k + 1) & 1];
        const int m = k + 1;  // this pass fills the region at margin m
        for (int i = threadIdx.x; i < RY * RX; i += 256) {
            const int ry = i / RX, rx = i % RX;
            if (ry < m || ry >= RY - m || rx < m || rx >= RX - m) continue;
            const int gy = gy0 + ry, gx = gx0 + rx;
            if (gy < 0 || gx < 0 || gy >= H - 1 || gx >= W - 1) {
                dst[i] = 0.f;
                continue;
            }
            float s = 0.f;
            for (int dy = -1; dy <= 1; ++dy) {
                const int yy = gy + dy;
                if (yy < 0 || yy >= H - 1) continue;
                for (int dx = -1; dx <= 1; ++dx) {
                    const int xx = gx + dx;
                    if (xx < 0 || xx >= W - 1) continue;
                    s += (float)((dy == 0 ? 2 : 1) * (dx == 0 ? 2 : 1)) * src[(ry + dy) * RX + rx + dx];
                }
            }
            dst[i] = s * (1.f / 16.f);
        }
        __syncthreads();
    }
    const float *res = buf[PASSES & 1];
    for (int i = threadIdx.x; i < kHeadY * kHeadX; i += 256) {
        const int gy = ty * kHeadY + i / kHeadX, gx = tx * kHeadX + i % kHeadX;
        if (gy < H && gx < W) out[img + (int64_t)gy * W + gx] = res[(i / kHeadX + PASSES) * RX + i % kHeadX + PASSES];
    }
}

// per (slice, sample): sums of t^2 and (y - t)^2 -> part[b][slice][2]
__global__ __launch_bounds__(256) void k_loss_part(const float *__restrict__ y, const float *__restrict__ t,
                                                   int64_t HW, int slices, double *__restrict__ part) {
    __shared__ double red[2 * 4];
    const int b = blockIdx.y, s = blockIdx.x;
    const int64_t per = (HW + slices - 1) / slices;
    const int64_t i0 = s * per, i1 = std::min<int64_t>(HW, i0 + per);
    double v[2] = {0.0, 0.0};
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const double tv = t[b * HW + i], dv = (double)y[b * HW + i] - tv;
        v[0] += tv * tv;
        v[1] += dv * dv;
    }
    block_sum_n<256, 2>(v, red);
    if (threadIdx.x == 0) {
        part[((int64_t)b * slices + s) * 2] = v[0];
        part[((int64_t)b * slices + s) * 2 + 1] = v[1];
    }
}

// sums[b] = (sum t^2, sum (y-t)^2); loss = mean over b of the ratio (one thread)
__global__ void k_loss_fin(const double *__restrict__ part, int B, int slices, double *__restrict__ sums,
                           double *__restrict__ loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double L = 0.0;
    for (int b = 0; b < B; ++b) {
        double st = 0.0, se = 0.0;
        for (int s = 0; s < slices; ++s) {
            st += part[((int64_t)b * slices + s) * 2];
            se += part[((int64_t)b * slices + s) * 2 + 1];
        }
        sums[2 * b] = st;
        sums[2 * b + 1] = se;
        L += se / fmax(st, 1e-300);
    }
    if (loss) *loss = L / B;
}

// Energy loss on the structured grid.  An image of n x n pixels holds the
// interior nodes of the unit square's n x n-cell grid, each cell cut by its
// diagonal from the lower-left to the upper-right corner: pixel (y, x) is node
// (x + 1, y + 1) and the last row and column hold no node.  With homogeneous
// Dirichlet data the P1 operator -Delta + nu I of eq. (4) on these nodes is the
// 5-point Laplacian plus nu h^2 times the P1 mass stencil (1/2 at the node,
// 1/12 at its six edge neighbours: the four axis neighbours and the two along
// the diagonal), h = 1 / n.
__device__ __forceinline__ double grid_op(const float *__restrict__ v, int n, int y, int x, double nuh2) {
    auto at = [&](int yy, int xx) -> double {
        return (yy >= 0 && xx >= 0 && yy < n - 1 && xx < n - 1) ? (double)v[(int64_t)yy * n + xx] : 0.0;
    };
    const double c = at(y, x), ax = at(y, x + 1) + at(y, x - 1) + at(y + 1, x) + at(y - 1, x),
                 dg = at(y + 1, x + 1) + at(y - 1, x - 1);
    return 4.0 * c - ax + nuh2 * (0.5 * c + (ax + dg) * (1.0 / 12.0));
}

__device__ __forceinline__ double sample_nuh2(const float *__restrict__ in2, int64_t HW, int b, int n, double nu_scale) {
    const double h = 1.0 / n;
    return nu_scale * (double)in2[(int64_t)b * HW * 2 + 1] * h * h;
}

// per (slice, sample) over interior pixels: y.At, y.Ay, t.At -> part[b][slice][3]
__global__ __launch_bounds__(256) void k_eloss_part(const float *__restrict__ y, const float *__restrict__ t,
                                                    const float *__restrict__ in2, int n, double nu_scale,
                                                    int slices, double *__restrict__ part) {
    __shared__ double red[3 * 4];
    const int b = blockIdx.y, s = blockIdx.x;
    const int64_t HW = (int64_t)n * n;
    const int64_t per = (HW + slices - 1) / slices;
    const int64_t i0 = s * per, i1 = std::min<int64_t>(HW, i0 + per);
    const double nuh2 = sample_nuh2(in2, HW, b, n, nu_scale);
    const float *yb = y + b * HW, *tb = t + b * HW;
    double v[3] = {0.0, 0.0, 0.0};
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const int py = (int)(i / n), px = (int)(i % n);
        if (py >= n - 1 || px >= n - 1) continue;
        const double At = grid_op(tb, n, py, px, nuh2), Ay = grid_op(yb, n, py, px, nuh2), yv = yb[i];
        v[0] += yv * At;
        v[1] += yv * Ay;
        v[2] += (double)tb[i] * At;
    }
    block_sum_n<256, 3>(v, red);
    if (threadIdx.x == 0)
        for (int k = 0; k < 3; ++k) part[((int64_t)b * slices + s) * 3 + k] = v[k];
}

// sums[b] = (y.At, y.Ay, t.At); loss = mean over b of 1 - (y.At)^2 / ((y.Ay)(t.At)),
// a sample with y.Ay <= 0 or t.At <= 0 counting 1 (one thread, fixed order)
__global__ void k_eloss_fin(const double *__restrict__ part, int B, int slices, double *__restrict__ sums,
                            double *__restrict__ loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double L = 0.0;
    for (int b = 0; b < B; ++b) {
        double v[3] = {0.0, 0.0, 0.0};
        for (int s = 0; s < slices; ++s)
            for (int k = 0; k < 3; ++k) v[k] += part[((int64_t)b * slices + s) * 3 + k];
        for (int k = 0; k < 3; ++k) sums[3 * b + k] = v[k];
        L += (v[1] > 0.0 && v[2] > 0.0) ? 1.0 - v[0] * v[0] / (v[1] * v[2]) : 1.0;
    }
    if (loss) *loss = L / B;
}

__device__ __forceinline__ void out_grad_store(float g, const float *__restrict__ w, int C, int64_t p, float *gy,
                                               bf16 *__restrict__ gd0) {
    gy[p] = g;
    if (!gd0) return;
    for (int c = 0; c < C; c += 8) {
        bf8 v;
#pragma unroll
        for (int i = 0; i < 8; ++i) v[i] = (bf16)(g * w[c + i]);
        *reinterpret_cast<bf8 *>(gd0 + p * C + c) = v;
    }
}

// gy = (1/B) (2 a^2 / (b^2 c) A y - 2 a / (b c) A t) on interior pixels, 0
// elsewhere (a, b, c = y.At, y.Ay, t.At); gd0[p][c] = gy w[c] (BF16)
__global__ void k_eloss_bwd(const float *__restrict__ y, const float *__restrict__ t, const float *__restrict__ in2,
                            const double *__restrict__ sums, const float *__restrict__ w, int C, int n, int B,
                            double nu_scale, float *__restrict__ gy, bf16 *__restrict__ gd0) {
    const int64_t HW = (int64_t)n * n, P = HW * B;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(p / HW);
        const int64_t i = p % HW;
        const int py = (int)(i / n), px = (int)(i % n);
        const double a = sums[3 * b], bb = sums[3 * b + 1], c = sums[3 * b + 2];
        double g = 0.0;
        if (py < n - 1 && px < n - 1 && bb > 0.0 && c > 0.0) {
            const double nuh2 = sample_nuh2(in2, HW, b, n, nu_scale);
            const double Ay = grid_op(y + b * HW, n, py, px, nuh2), At = grid_op(t + b * HW, n, py, px, nuh2);
            g = (2.0 * a / (bb * c)) * (a / bb * Ay - At) / B;
        }
        out_grad_store((float)g, w, C, p, gy, gd0);
    }
}

// Output smoothing: one pass of the 3x3 binomial filter (1 2 1; 2 4 2; 1 2 1) / 16
// over the pixels x < W-1, y < H-1 of each image, the last row and column read
// and written as 0 (they hold no node in the grid layout).  As a matrix the
// pass is M K M with K the zero-padded symmetric convolution and M that pixel
// mask, so it is symmetric and serves as its own adjoint in the backward pass.
__global__ void k_binom(const float *__restrict__ in, int H, int W, int64_t P, float *__restrict__ out) {
    const int64_t HW = (int64_t)H * W;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = p % HW;
        const int y = (int)(i / W), x = (int)(i % W);
        if (y >= H - 1 || x >= W - 1) {
            out[p] = 0.f;
            continue;
        }
        const float *im = in + (p - i);
        float s = 0.f;
        for (int dy = -1; dy <= 1; ++dy) {
            const int yy = y + dy;
            if (yy < 0 || yy >= H - 1) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                const int xx = x + dx;
                if (xx < 0 || xx >= W - 1) continue;
                s += (float)((dy == 0 ? 2 : 1) * (dx == 0 ? 2 : 1)) * im[(int64_t)yy * W + xx];
            }
        }
        out[p] = s * (1.f / 16.f);
    }
}

// gd0[p][c] = gy[p] w[c] (BF16)
__global__ void k_out_gd0(const float *__restrict__ gy, const float *__restrict__ w, int C, int64_t P,
                          bf16 *__restrict__ gd0) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        const float g = gy[p];
        for (int c = 0; c < C; c += 8) {
            bf8 v;
#pragma unroll
            for (int i = 0; i < 8; ++i) v[i] = (bf16)(g * w[c + i]);
            *reinterpret_cast<bf8 *>(gd0 + p * C + c) = v;
        }
    }
}

// gy = 2 (y - t) / (B sum t^2) (FP32), gd0[p][c] = gy w[c] (BF16; skipped when gd0 is NULL)
__global__ void k_out_bwd(const float *__restrict__ y, const float *__restrict__ t, const double *__restrict__ sums,
                          const float *__restrict__ w, int C, int64_t HW, int B, float *__restrict__ gy,
                          bf16 *__restrict__ gd0) {
    const int64_t P = HW * B;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = p / HW;
        const float g = (float)(2.0 * ((double)y[p] - t[p]) / ((double)B * fmax(sums[2 * b], 1e-300)));
        out_grad_store(g, w, C, p, gy, gd0);
    }
}

// 1x1 output layer weight gradient over pixel slices:
// part[s][c] = sum_p d0[p][c] gy[p] (c < C), part[s][C] = sum_p gy[p].  Each
// thread accumulates all C + 1 sums over its pixels (16-byte loads of 8
// channels), then one block reduction of all of them (fixed order).
template <int C>
__global__ __launch_bounds__(256) void k_out_wgrad(const bf16 *__restrict__ d0, const float *__restrict__ gy,
                                                   int64_t P, float *__restrict__ part) {
    __shared__ double red[(C + 1) * 4];
    const int s = blockIdx.x;
    const int64_t p0 = (int64_t)s * kWSlice, p1 = std::min<int64_t>(P, p0 + kWSlice);
    double v[C + 1];
#pragma unroll
    for (int c = 0; c <= C; ++c) v[c] = 0.0;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += 256) {
        const double g = (double)gy[p];
#pragma unroll
        for (int c8 = 0; c8 < C; c8 += 8) {
            const bf8 a = ld8(d0 + p * C + c8);
#pragma unroll
            for (int i = 0; i < 8; ++i) v[c8 + i] += g * (double)(float)a[i];
        }
        v[C] += g;
    }
    block_sum_n<256, C + 1>(v, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c <= C; ++c) part[(int64_t)s * (C + 1) + c] = (float)v[c];
}

// Adam on the FP32 master weights; c1, c2 are the bias corrections 1 - beta^t
__global__ void k_adam(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// B operands in fragment order from the FP32 weights.
struct MapConvFwd {  // k = tap*Cin + ci, n = co: W[tap][ci][co]
    const float *w;
    int Cin, Cout;
    __device__ float operator()(int k, int n) const { return k < 9 * Cin ? w[(int64_t)k * Cout + n] : 0.f; }
};
struct MapConvBwd {  // k = tap*Cout + co, n = ci: W[8 - tap][ci][co] (the transposed convolution's taps)
    const float *w;
    int Cin, Cout;
    __device__ float operator()(int k, int n) const {
        const int tap = k / Cout, co = k - tap * Cout;
        if (tap >= 9 || n >= Cin) return 0.f;
        return w[((int64_t)(8 - tap) * Cin + n) * Cout + co];
    }
};
struct MapUpFwd {  // k = ci, n = q*Cout + co: W[ci][q][co]
    const float *w;
    int Cin, Cout;
    __device__ float operator()(int k, int n) const { return k < Cin ? w[(int64_t)k * 4 * Cout + n] : 0.f; }
};
struct MapUpBwd {  // k = q*Cout + co, n = ci: W[ci][q][co]
    const float *w;
    int Cin, Cout;
    __device__ float operator()(int k, int n) const {
        return (k < 4 * Cout && n < Cin) ? w[(int64_t)n * 4 * Cout + k] : 0.f;
    }
};
template <class Map>
__global__ void k_pack_b(Map map, int KB, int NT, bf16 *__restrict__ Bp) {
    const int64_t total = (int64_t)KB * NT * 64 * 8;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int e = (int)(i % 8);
        int64_t t = i / 8;
        const int lane = (int)(t % 64);
        t /= 64;
        const int nt = (int)(t % NT);
        const int kb = (int)(t / NT);
        Bp[i] = (bf16)map(kb * 32 + 8 * (lane >> 4) + e, nt * 16 + (lane & 15));
    }
}

// ---------------------------------------------------------------------------
// Grid glue of the preconditioner: nodal residual -> image, image -> nodal z.
// Node (i, j) of the (N+1) x (N+1) grid is i + j (N+1); interior node (i, j),
// 1 <= i, j <= N-1, is pixel (x, y) = (i-1, j-1) of an N x N image whose last
// row and column are zero padding.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_interior_sumsq(const double *__restrict__ r, int N, double *__restrict__ part) {
    __shared__ double red[4];
    const int64_t n = (int64_t)(N - 1) * (N - 1);
    double s = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
        const int64_t x = p % (N - 1), y = p / (N - 1);
        const double v = r[(y + 1) * (N + 1) + x + 1];
        s += v * v;
    }
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}
// inv[0] = 1 / RMS over the (N-1)^2 interior values from the per-block sums of
// squares (fixed order), 0 for a zero vector
__global__ __launch_bounds__(256) void k_grid_scale(const double *__restrict__ part, int nparts, int N,
                                                    double *__restrict__ inv) {
    __shared__ double red[4];
    double s = 0.0;
    for (int k = threadIdx.x; k < nparts; k += 256) s += part[k];
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) {
        const double n_int = (double)(N - 1) * (N - 1);
        inv[0] = s > 0.0 ? 1.0 / sqrt(s / n_int) : 0.0;
    }
}
// network input: pixel (x, y) <- interior node (x + 1, y + 1) scaled by inv[0];
// last row and column 0; channel 1 = cval
__global__ void k_grid_in(const double *__restrict__ r, const double *__restrict__ inv_p, int N, float cval,
                          float *__restrict__ in2) {
    const double inv = inv_p[0];
    const int64_t P = (int64_t)N * N;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(p % N), y = (int)(p / N);
        float v = 0.f;
        if (x < N - 1 && y < N - 1) v = (float)(r[(int64_t)(y + 1) * (N + 1) + (x + 1)] * inv);
        in2[2 * p] = v;
        in2[2 * p + 1] = cval;
    }
}
// FP32 -> BF16 rounding to nearest even, written on the bits: the conversion
// the (bf16) cast performs on finite values, but as integer operations on the
// stored FP32 value, so that it cannot be merged with a preceding FP64 -> FP32
// rounding (one rounding from FP64 can differ from the two).  NaN: the cast.
__device__ __forceinline__ bf16 bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16)f;
    const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    return __builtin_bit_cast(bf16, (uint16_t)(r >> 16));
}
// k_grid_in and k_make_input in one pass: the network's BF16 input (8
// channels, 2 used) of the scaled interior residual, the values k_make_input
// forms from k_grid_in's FP32 image
__global__ void k_grid_in8(const double *__restrict__ r, const double *__restrict__ inv_p, int N, float cval,
                           bf16 *__restrict__ x8) {
    const double inv = inv_p[0];
    const int64_t P = (int64_t)N * N;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(p % N), y = (int)(p / N);
        float v = 0.f;
        if (x < N - 1 && y < N - 1) v = (float)(r[(int64_t)(y + 1) * (N + 1) + (x + 1)] * inv);
        bf8 o = zero8();
        o[0] = bf16_rne(v);
        o[1] = bf16_rne(cval);
        *reinterpret_cast<bf8 *>(x8 + p * 8) = o;
    }
}
// e = u - x on the interior: per-block sums of squares
__global__ __launch_bounds__(256) void k_interior_sumsq_diff(const double *__restrict__ u, const double *__restrict__ x,
                                                             int N, double *__restrict__ part) {
    __shared__ double red[4];
    const int64_t n = (int64_t)(N - 1) * (N - 1);
    double s = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n; p += (int64_t)gridDim.x * 256) {
        const int64_t g = (p / (N - 1) + 1) * (N + 1) + p % (N - 1) + 1;
        const double v = u[g] - x[g];
        s += v * v;
    }
    s = block_sum<256>(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}
// training target: pixel (x, y) <- (u - x) at interior node (x + 1, y + 1) scaled by inv[0]
__global__ void k_grid_target(const double *__restrict__ u, const double *__restrict__ xv,
                              const double *__restrict__ inv_p, int N, float *__restrict__ t) {
    const double inv = inv_p[0];
    const int64_t P = (int64_t)N * N;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(p % N), y = (int)(p / N);
        float v = 0.f;
        if (x < N - 1 && y < N - 1) {
            const int64_t g = (int64_t)(y + 1) * (N + 1) + (x + 1);
            v = (float)((u[g] - xv[g]) * inv);
        }
        t[p] = v;
    }
}
__global__ void k_grid_out(const float *__restrict__ out, int N, const uint8_t *__restrict__ mask, double *__restrict__ z) {
    const int64_t n = (int64_t)(N + 1) * (N + 1);
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(g % (N + 1)), j = (int)(g / (N + 1));
        double v = 0.0;
        if (i >= 1 && i <= N - 1 && j >= 1 && j <= N - 1) v = out[(int64_t)(j - 1) * N + (i - 1)];
        if (mask && mask[g]) v = 0.0;
        z[g] = v;
    }
}

// slots of UNet::gpart: [0, 1024) and [1024, 2048) per-block sums, then the scales
constexpr int kGridScale = 2048;

inline int grid1(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384)); }

enum LayerKind { CONV = 0, UP = 1 };

struct Layer {
    int kind;
    int lvl;     // level of the GEMM rows (conv: its level; up-conv: the low level)
    int C1, C2;  // input channels (conv: concatenation split; up-conv: C1 = Cin)
    int Cout;
    int64_t woff, boff;
    bf16 *Bf = nullptr, *Bb = nullptr;
    int KBf = 0, NTf = 0, KBb = 0, NTb = 0;
    int Cin() const { return C1 + C2; }
};

struct Tensor {
    bf16 *a = nullptr, *g = nullptr;
    int lvl = 0, C = 0;
};

}  // namespace

struct UNet {
    int H = 0, W = 0, maxB = 0, c = 0;
    std::vector<Layer> L;
    int64_t nparam = 0, out_woff = 0, out_boff = 0;
    int64_t step = 0;
    void *arena = nullptr;
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    Tensor x8, e0a, e0, p0, e1a, e1, p1, e2a, e2, p2, ma, mm, u2, d2a, d2, u1, d1a, d1, u0, d0a, d0;
    float *out = nullptr, *gy = nullptr, *partial = nullptr;
    double *sums = nullptr, *lpart = nullptr, *gpart = nullptr;
    int64_t partial_cap = 0;
    int loss_slices = 64;
    int loss_kind = FEM_UNET_LOSS_L2;
    double nu_scale = 0.0;  // energy loss: nu = nu_scale * input channel 1
    int out_smooth = 0;     // binomial passes on the output
    float *ys = nullptr;    // their second buffer
};

namespace {

int64_t pixels(const UNet &N, int lvl, int B) { return (int64_t)B * (N.H >> lvl) * (N.W >> lvl); }

template <class Src, class Epi>
int launch_rows(const Src &s, const Epi &e, const bf16 *Bp, int64_t M, int KB, int NT, hipStream_t st) {
    const int g = (int)((M + kPixTile - 1) / kPixTile);
    const int m = (int)M;
    switch (NT) {
        case 1: k_gemm_rows<Src, Epi, 1><<<g, 256, 0, st>>>(s, e, Bp, m, KB); break;
        case 2: k_gemm_rows<Src, Epi, 2><<<g, 256, 0, st>>>(s, e, Bp, m, KB); break;
        case 4: k_gemm_rows<Src, Epi, 4><<<g, 256, 0, st>>>(s, e, Bp, m, KB); break;
        case 8: k_gemm_rows<Src, Epi, 8><<<g, 256, 0, st>>>(s, e, Bp, m, KB); break;
        case 16: k_gemm_rows<Src, Epi, 16><<<g, 256, 0, st>>>(s, e, Bp, m, KB); break;
        case 32: k_gemm_rows<Src, Epi, 32><<<g, 256, 0, st>>>(s, e, Bp, m, KB); break;
        default: return set_error(FEM_EINVAL, "unsupported GEMM width");
    }
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

int64_t wgrad_splits(int64_t P, int64_t slice = kWSlice) { return std::max<int64_t>(1, (P + slice - 1) / slice); }

// Pixels per weight-gradient slice of a GEMM with R1 rows: kWSlice, halved
// (down to 128, a multiple of k_wgrad_conv's chunk) while the launch would
// have fewer than kWGradTarget workgroups, so that the coarse levels, whose
// operands are gathered with long latency chains, fill the GPU.
constexpr int kWGradTarget = 1024;
int64_t wgrad_slice(int64_t P, int R1, int rows_per_block = 64) {
    const int64_t rb = (R1 + rows_per_block - 1) / rows_per_block;
    int64_t s = kWSlice;
    while (s > 128 && wgrad_splits(P, s) * rb < kWGradTarget) s /= 2;
    return s;
}

// im2col rows per workgroup of k_wgrad_conv for NT output column tiles: two
// row tiles per wave for 64 output channels (their layers have 289-1153 rows,
// and the staged gradient serves twice the MFMAs; 52 KiB of static LDS);
// measured slower for 16 and 32 channels (fewer rows to share it, lower
// occupancy), and 128 channels would exceed 64 KiB
inline int conv_wgrad_rows(int NT) { return NT == 4 ? 128 : 64; }

// launches the weight-gradient GEMM; *splits receives its slice count
template <class WS, class WG>
int launch_wgrad(UNet &N, const WS &ws, const WG &wg, int R1, int Nc, int64_t P, int64_t *splits_out,
                 hipStream_t st) {
    const int64_t slice = wgrad_slice(P, R1);
    const int64_t splits = wgrad_splits(P, slice);
    if (splits * R1 * Nc > N.partial_cap || splits > 65535)
        return set_error(FEM_EINVAL, "weight-gradient scratch too small");
    *splits_out = splits;
    const int NT = (Nc + 15) / 16;
    const unsigned grid = wgrad_grid((R1 + 63) / 64, splits);
    switch (NT) {
        case 1: k_gemm_wgrad<WS, WG, 1><<<grid, 256, 0, st>>>(ws, wg, R1, Nc, P, slice, N.partial); break;
        case 2: k_gemm_wgrad<WS, WG, 2><<<grid, 256, 0, st>>>(ws, wg, R1, Nc, P, slice, N.partial); break;
        case 4: k_gemm_wgrad<WS, WG, 4><<<grid, 256, 0, st>>>(ws, wg, R1, Nc, P, slice, N.partial); break;
        case 8: k_gemm_wgrad<WS, WG, 8><<<grid, 256, 0, st>>>(ws, wg, R1, Nc, P, slice, N.partial); break;
        case 16: k_gemm_wgrad<WS, WG, 16><<<grid, 256, 0, st>>>(ws, wg, R1, Nc, P, slice, N.partial); break;
        case 32: k_gemm_wgrad<WS, WG, 32><<<grid, 256, 0, st>>>(ws, wg, R1, Nc, P, slice, N.partial); break;
        default: return set_error(FEM_EINVAL, "unsupported GEMM width");
    }
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

int repack(UNet &N, hipStream_t st) {
    for (auto &l : N.L) {
        const float *w = N.w + l.woff;
        const int64_t nf = (int64_t)l.KBf * l.NTf * 512, nb = (int64_t)l.KBb * l.NTb * 512;
        if (l.kind == CONV) {
            k_pack_b<<<grid1(nf), 256, 0, st>>>(MapConvFwd{w, l.Cin(), l.Cout}, l.KBf, l.NTf, l.Bf);
            if (l.Bb) k_pack_b<<<grid1(nb), 256, 0, st>>>(MapConvBwd{w, l.Cin(), l.Cout}, l.KBb, l.NTb, l.Bb);
        } else {
            k_pack_b<<<grid1(nf), 256, 0, st>>>(MapUpFwd{w, l.C1, l.Cout}, l.KBf, l.NTf, l.Bf);
            k_pack_b<<<grid1(nb), 256, 0, st>>>(MapUpBwd{w, l.C1, l.Cout}, l.KBb, l.NTb, l.Bb);
        }
    }
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

size_t conv_lds(int TY, int TX, int Cin, int KB, int NT) { return conv_lds_bytes(TY, TX, Cin, KB, NT); }

// the tiled kernel takes power-of-two channel counts from 8 to 128 whose tile
// and weight block fit in 64 KiB of LDS (at least two workgroups per CU)
bool conv_tile_fits(int TY, int TX, const Layer &l) {
    const int c = l.Cin();
    return c >= 8 && c <= 128 && (c & (c - 1)) == 0 && conv_lds(TY, TX, c, l.KBf, l.NTf) <= 65536;
}

// Tiles of fewer workgroups than twice the CU count (the coarsest level at
// batch 1: 256 tiles of 64 pixels) split their output channels over two
// workgroups when each keeps at least four column tiles: twice the
// workgroups, each with half the weight stages.
template <int TY, int TX, int NT, int CIN>
int launch_conv3x3(UNet &N, const Layer &l, const Tensor &s1, const Tensor *s2, const Tensor &y, int B,
                   hipStream_t st, const Tensor *pool = nullptr, bool *pooled = nullptr) {
    const int H = N.H >> l.lvl, W = N.W >> l.lvl;
    const int tiles_x = (W + TX - 1) / TX, tiles_y = (H + TY - 1) / TY;
    const int64_t tiles = (int64_t)B * tiles_x * tiles_y;
    // with a pooled output: the pooling in the epilogue when the tile's outputs
    // fit where its input was staged
    if constexpr (TY % 2 == 0 && TX % 2 == 0 && NT <= 4) {
        if (pool && pooled && conv_tile_bytes(TY, TX, CIN) >= (size_t)TY * TX * NT * 16 * 2) {
            const size_t lds = conv_lds(TY, TX, CIN, l.KBf, NT);
            k_conv3x3<TY, TX, NT, CIN, 1, false, true><<<(unsigned)tiles, 256, lds, st>>>(
                s1.a, s2 ? s2->a : nullptr, l.C1, H, W, tiles_x, tiles_y, l.Bf, N.w + l.boff, y.a, pool->a, 0);
            FEM_HIP_CHECK(hipGetLastError());
            *pooled = true;
            return 0;
        }
    }
    if constexpr (NT >= 8) {
        if (tiles < 2 * device_cu_count()) {
            const size_t lds = conv_lds(TY, TX, CIN, l.KBf, NT / 2);
            k_conv3x3<TY, TX, NT, CIN, 2><<<(unsigned)(2 * tiles), 256, lds, st>>>(
                s1.a, s2 ? s2->a : nullptr, l.C1, H, W, tiles_x, tiles_y, l.Bf, N.w + l.boff, y.a, nullptr, 0);
            FEM_HIP_CHECK(hipGetLastError());
            return 0;
        }
    }
    const size_t lds = conv_lds(TY, TX, CIN, l.KBf, NT);
    k_conv3x3<TY, TX, NT, CIN><<<(unsigned)tiles, 256, lds, st>>>(s1.a, s2 ? s2->a : nullptr, l.C1, H, W, tiles_x,
                                                                   tiles_y, l.Bf, N.w + l.boff, y.a, nullptr, 0);
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

// CIN of the layer as a template constant (conv_tile_fits has checked it)
template <int TY, int TX, int NT>
int launch_conv_cin(UNet &N, const Layer &l, const Tensor &s1, const Tensor *s2, const Tensor &y, int B,
                    hipStream_t st, const Tensor *pool = nullptr, bool *pooled = nullptr) {
    switch (l.Cin()) {
        case 8: return launch_conv3x3<TY, TX, NT, 8>(N, l, s1, s2, y, B, st, pool, pooled);
        case 16: return launch_conv3x3<TY, TX, NT, 16>(N, l, s1, s2, y, B, st, pool, pooled);
        case 32: return launch_conv3x3<TY, TX, NT, 32>(N, l, s1, s2, y, B, st, pool, pooled);
        case 64:
            if constexpr ((TY + 2) * (TX + 2) * 64 * 2 <= 49152)
                return launch_conv3x3<TY, TX, NT, 64>(N, l, s1, s2, y, B, st, pool, pooled);
            break;
        case 128:
            if constexpr ((TY + 2) * (TX + 2) * 128 * 2 <= 49152)
                return launch_conv3x3<TY, TX, NT, 128>(N, l, s1, s2, y, B, st, pool, pooled);
            break;
        default: break;
    }
    return set_error(FEM_EINVAL, "internal error: no tiled convolution for this channel count");
}

// forward conv3x3 + ReLU: 8 x 32 pixel tiles (4 row tiles per wave) on the two
// fine levels (16 x 32 for 32 output channels), 4 x 16 on the coarse ones,
// each where its input tile fits the LDS budget; otherwise the row GEMM
// reading the input directly
// (pool, pooled: when the tiled kernel runs with the layer's 2 x 2 average
// pooling into pool in its epilogue, *pooled is set)
int conv_fwd(UNet &N, const Layer &l, const Tensor &s1, const Tensor *s2, const Tensor &y, int B, hipStream_t st,
             const Tensor *pool = nullptr, bool *pooled = nullptr) {
    // 32 output channels: 16 x 32 tiles (8 row tiles per wave) where the input
    // tile fits (measured 41.6 us against 49.6 us for 8 x 32 at 512^2; with 16
    // output channels the taller tile was slower, 81 against 70 us at 1024^2)
    if (l.lvl <= 1 && l.NTf == 2 && conv_tile_fits(16, 32, l))
        return launch_conv_cin<16, 32, 2>(N, l, s1, s2, y, B, st, pool, pooled);
    if (l.lvl <= 1 && conv_tile_fits(8, 32, l)) {
        switch (l.NTf) {
            case 1: return launch_conv_cin<8, 32, 1>(N, l, s1, s2, y, B, st, pool, pooled);
            case 2: return launch_conv_cin<8, 32, 2>(N, l, s1, s2, y, B, st, pool, pooled);
            case 4: return launch_conv_cin<8, 32, 4>(N, l, s1, s2, y, B, st, pool, pooled);
            default: break;
        }
    }
    if (conv_tile_fits(4, 16, l)) {
        switch (l.NTf) {
            case 1: return launch_conv_cin<4, 16, 1>(N, l, s1, s2, y, B, st, pool, pooled);
            case 2: return launch_conv_cin<4, 16, 2>(N, l, s1, s2, y, B, st, pool, pooled);
            case 4: return launch_conv_cin<4, 16, 4>(N, l, s1, s2, y, B, st, pool, pooled);
            case 8: return launch_conv_cin<4, 16, 8>(N, l, s1, s2, y, B, st);
            case 16: return launch_conv_cin<4, 16, 16>(N, l, s1, s2, y, B, st);
            default: break;
        }
    }
    SrcConv src{s1.a, s2 ? s2->a : nullptr, l.C1, l.C2, N.H >> l.lvl, N.W >> l.lvl};
    EpiConv epi{y.a, N.w + l.boff, l.Cout};
    return launch_rows(src, epi, l.Bf, pixels(N, l.lvl, B), l.KBf, l.NTf, st);
}

// Input gradient of a 3x3 convolution through the LDS-tiled kernel: the
// convolution, with the flipped packed weights Bb, of the output gradient
// masked by the layer's ReLU (CO = Cout staged channels, NT = Cin / 16 output
// column tiles, split over s1.g and s2->g at C1).
template <int TY, int TX, int NT, int CO>
int launch_conv_bwd3x3(UNet &N, const Layer &l, const Tensor &s1, const Tensor *s2, const Tensor &y, int B,
                       hipStream_t st) {
    const int H = N.H >> l.lvl, W = N.W >> l.lvl;
    const int tiles_x = (W + TX - 1) / TX, tiles_y = (H + TY - 1) / TY;
    const int64_t tiles = (int64_t)B * tiles_x * tiles_y;
    const size_t lds = conv_lds(TY, TX, CO, l.KBb, NT);
    k_conv3x3<TY, TX, NT, CO, 1, true><<<(unsigned)tiles, 256, lds, st>>>(
        y.g, y.a, CO, H, W, tiles_x, tiles_y, l.Bb, nullptr, s1.g, s2 ? s2->g : nullptr, l.C1);
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

template <int TY, int TX, int NT>
int launch_conv_bwd_co(UNet &N, const Layer &l, const Tensor &s1, const Tensor *s2, const Tensor &y, int B,
                       hipStream_t st) {
    switch (l.Cout) {
        case 16: return launch_conv_bwd3x3<TY, TX, NT, 16>(N, l, s1, s2, y, B, st);
        case 32: return launch_conv_bwd3x3<TY, TX, NT, 32>(N, l, s1, s2, y, B, st);
        case 64:
            if constexpr ((TY + 2) * (TX + 2) * 64 * 2 <= 49152) return launch_conv_bwd3x3<TY, TX, NT, 64>(N, l, s1, s2, y, B, st);
            break;
        case 128:
            if constexpr ((TY + 2) * (TX + 2) * 128 * 2 <= 49152)
                return launch_conv_bwd3x3<TY, TX, NT, 128>(N, l, s1, s2, y, B, st);
            break;
        default: break;
    }
    return 1;
}

// 1 when the tiled kernel does not apply (the row GEMM takes the layer)
int conv_bwd_data_tiled(UNet &N, const Layer &l, const Tensor &s1, const Tensor *s2, const Tensor &y, int B,
                        hipStream_t st) {
    const int Cin = l.Cin(), co = l.Cout;
    if (Cin % 16 || l.C1 % 16 || co < 16 || co > 128 || (co & (co - 1)) || l.NTb * 16 != Cin) return 1;
    auto fits = [&](int TY, int TX) { return conv_lds(TY, TX, co, l.KBb, l.NTb) <= 65536; };
    if (l.lvl <= 1 && fits(8, 32)) {
        switch (l.NTb) {
            case 1: return launch_conv_bwd_co<8, 32, 1>(N, l, s1, s2, y, B, st);
            case 2: return launch_conv_bwd_co<8, 32, 2>(N, l, s1, s2, y, B, st);
            case 4: return launch_conv_bwd_co<8, 32, 4>(N, l, s1, s2, y, B, st);
            default: break;
        }
    }
    if (fits(4, 16)) {
        switch (l.NTb) {
            case 1: return launch_conv_bwd_co<4, 16, 1>(N, l, s1, s2, y, B, st);
            case 2: return launch_conv_bwd_co<4, 16, 2>(N, l, s1, s2, y, B, st);
            case 4: return launch_conv_bwd_co<4, 16, 4>(N, l, s1, s2, y, B, st);
            case 8: return launch_conv_bwd_co<4, 16, 8>(N, l, s1, s2, y, B, st);
            default: break;
        }
    }
    return 1;
}

// conv3x3 + ReLU backward: input gradients into s1.g (and s2->g), overwritten; weight gradients
int conv_bwd(UNet &N, const Layer &l, const Tensor &s1, const Tensor *s2, const Tensor &y, bool input_grad, int B,
             hipStream_t st) {
    const int H = N.H >> l.lvl, W = N.W >> l.lvl;
    const int64_t M = pixels(N, l.lvl, B);
    if (input_grad) {
        if (l.Cout & (l.Cout - 1)) return set_error(FEM_EINVAL, "output channel count must be a power of two");
        const int rt = conv_bwd_data_tiled(N, l, s1, s2, y, B, st);
        if (rt < 0) return rt;
        if (rt == 1) {
            SrcConvBwd src{y.g, y.a, l.Cout, __builtin_ctz((unsigned)l.Cout), H, W};
            EpiGrad epi{s1.g, s2 ? s2->g : nullptr, l.C1, l.C2};
            if (int rc = launch_rows(src, epi, l.Bb, M, l.KBb, l.NTb, st)) return rc;
        }
    }
    const int R = 9 * l.Cin();
    WSrcConv ws{s1.a, s2 ? s2->a : nullptr, l.C1, l.C2, H, W, R};
    WGradConv wg{y.g, y.a, l.Cout};
    const int NTw = l.Cout / 16;
    int64_t splits = 0;
    if (l.C1 % 8 == 0 && l.C2 % 8 == 0 && l.Cout % 16 == 0 && (NTw == 1 || NTw == 2 || NTw == 4 || NTw == 8)) {
        const int rpb = conv_wgrad_rows(NTw);
        const int64_t slice = wgrad_slice(M, R + 1, rpb);
        splits = wgrad_splits(M, slice);
        if (splits * (R + 1) * l.Cout > N.partial_cap || splits > 65535)
            return set_error(FEM_EINVAL, "weight-gradient scratch too small");
        const unsigned grid = wgrad_grid((R + 1 + rpb - 1) / rpb, splits);
        switch (NTw) {
            case 1: k_wgrad_conv<1, 1><<<grid, 256, 0, st>>>(ws, wg, R + 1, l.Cout, M, slice, N.partial); break;
            case 2: k_wgrad_conv<2, 1><<<grid, 256, 0, st>>>(ws, wg, R + 1, l.Cout, M, slice, N.partial); break;
            case 4: k_wgrad_conv<4, 2><<<grid, 256, 0, st>>>(ws, wg, R + 1, l.Cout, M, slice, N.partial); break;
            default: k_wgrad_conv<8, 1><<<grid, 256, 0, st>>>(ws, wg, R + 1, l.Cout, M, slice, N.partial); break;
        }
        FEM_HIP_CHECK(hipGetLastError());
    } else if (int rc = launch_wgrad(N, ws, wg, R + 1, l.Cout, M, &splits, st)) {
        return rc;
    }
    const int64_t n = (int64_t)(R + 1) * l.Cout;  // weights [tap][ci][co] then the bias: contiguous
    k_sum_splits<<<grid1(n * kSumLanes), 256, 0, st>>>(N.partial, (int)splits, n, N.g + l.woff);
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

int up_fwd(UNet &N, const Layer &l, const Tensor &in, const Tensor &y, int B, hipStream_t st) {
    const int64_t M = pixels(N, l.lvl, B);
    const int H = N.H >> l.lvl, W = N.W >> l.lvl;
    auto pow2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
    if (l.Cout >= 16 && pow2(l.Cout) && pow2(H) && pow2(W) && M < ((int64_t)1 << 31)) {
        const int g = (int)((M + kPixTile - 1) / kPixTile);
        const int lc = __builtin_ctz((unsigned)l.Cout), lh = __builtin_ctz((unsigned)H), lw = __builtin_ctz((unsigned)W);
        const float *bias = N.w + l.boff;
        switch (l.NTf) {
            case 4: k_upconv<4><<<g, 256, 0, st>>>(in.a, l.C1, lc, lh, lw, (int)M, l.Bf, l.KBf, bias, y.a); break;
            case 8: k_upconv<8><<<g, 256, 0, st>>>(in.a, l.C1, lc, lh, lw, (int)M, l.Bf, l.KBf, bias, y.a); break;
            case 16: k_upconv<16><<<g, 256, 0, st>>>(in.a, l.C1, lc, lh, lw, (int)M, l.Bf, l.KBf, bias, y.a); break;
            case 32: k_upconv<32><<<g, 256, 0, st>>>(in.a, l.C1, lc, lh, lw, (int)M, l.Bf, l.KBf, bias, y.a); break;
            default: return set_error(FEM_EINVAL, "unsupported up-convolution width");
        }
        FEM_HIP_CHECK(hipGetLastError());
        return 0;
    }
    SrcRows src{in.a, l.C1};
    EpiUp epi{y.a, N.w + l.boff, l.Cout, N.H >> l.lvl, N.W >> l.lvl};
    return launch_rows(src, epi, l.Bf, M, l.KBf, l.NTf, st);
}

int up_bwd(UNet &N, const Layer &l, const Tensor &in, const Tensor &y, int B, hipStream_t st) {
    const int H = N.H >> l.lvl, W = N.W >> l.lvl;
    const int64_t M = pixels(N, l.lvl, B);
    SrcUpBwd src{y.g, l.Cout, H, W};
    EpiGrad epi{in.g, nullptr, l.C1, 0};
    if (int rc = launch_rows(src, epi, l.Bb, M, l.KBb, l.NTb, st)) return rc;
    WSrcUp ws{in.a, l.C1};
    WGradUp wg{y.g, l.Cout, H, W};
    int64_t splits = 0;
    if (int rc = launch_wgrad(N, ws, wg, l.C1 + 1, 4 * l.Cout, M, &splits, st)) return rc;
    const int64_t n = (int64_t)l.C1 * 4 * l.Cout + l.Cout;
    k_sum_splits_up<<<grid1(n * kSumLanes), 256, 0, st>>>(N.partial, (int)splits, l.C1, l.Cout, N.g + l.woff);
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

int pool(const UNet &N, const Tensor &in, const Tensor &out, int B, hipStream_t st) {
    const int H = N.H >> in.lvl, W = N.W >> in.lvl;
    k_pool_fwd<<<grid1(pixels(N, out.lvl, B) * (in.C / 8)), 256, 0, st>>>(in.a, out.a, B, H, W, in.C);
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

int pool_bwd(const UNet &N, const Tensor &in, const Tensor &out, int B, hipStream_t st) {
    const int H = N.H >> in.lvl, W = N.W >> in.lvl;
    k_pool_bwd<<<grid1(pixels(N, in.lvl, B) * (in.C / 8)), 256, 0, st>>>(out.g, in.g, B, H, W, in.C);
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

// forward of input [B][H][W][2] (FP32) into N.out [B][H][W]
// forward from the BF16 input already in N.x8
int forward_x8(UNet &N, int B, hipStream_t st) {
    const int64_t P0 = pixels(N, 0, B);
    const auto &L = N.L;
    int rc = 0;
    auto ok = [&](int r) {
        if (!rc) rc = r;
    };
    ok(conv_fwd(N, L[0], N.x8, nullptr, N.e0a, B, st));
    bool pooled = false;
    ok(conv_fwd(N, L[1], N.e0a, nullptr, N.e0, B, st, &N.p0, &pooled));
    if (!pooled) ok(pool(N, N.e0, N.p0, B, st));
    ok(conv_fwd(N, L[2], N.p0, nullptr, N.e1a, B, st));
    pooled = false;
    ok(conv_fwd(N, L[3], N.e1a, nullptr, N.e1, B, st, &N.p1, &pooled));
    if (!pooled) ok(pool(N, N.e1, N.p1, B, st));
    ok(conv_fwd(N, L[4], N.p1, nullptr, N.e2a, B, st));
    pooled = false;
    ok(conv_fwd(N, L[5], N.e2a, nullptr, N.e2, B, st, &N.p2, &pooled));
    if (!pooled) ok(pool(N, N.e2, N.p2, B, st));
    ok(conv_fwd(N, L[6], N.p2, nullptr, N.ma, B, st));
    ok(conv_fwd(N, L[7], N.ma, nullptr, N.mm, B, st));
    ok(up_fwd(N, L[8], N.mm, N.u2, B, st));
    ok(conv_fwd(N, L[9], N.u2, &N.e2, N.d2a, B, st));
    ok(conv_fwd(N, L[10], N.d2a, nullptr, N.d2, B, st));
    ok(up_fwd(N, L[11], N.d2, N.u1, B, st));
    ok(conv_fwd(N, L[12], N.u1, &N.e1, N.d1a, B, st));
    ok(conv_fwd(N, L[13], N.d1a, nullptr, N.d1, B, st));
    ok(up_fwd(N, L[14], N.d1, N.u0, B, st));
    ok(conv_fwd(N, L[15], N.u0, &N.e0, N.d0a, B, st));
    ok(conv_fwd(N, L[16], N.d0a, nullptr, N.d0, B, st));
    if (rc) return rc;
    if (N.out_smooth >= 1 && N.out_smooth <= 3) {
        const int tx = (N.W + kHeadX - 1) / kHeadX, ty = (N.H + kHeadY - 1) / kHeadY;
        const unsigned g = (unsigned)((int64_t)B * tx * ty);
        const float *wo = N.w + N.out_woff, *bo = N.w + N.out_boff;
        switch (N.out_smooth) {
            case 1: k_out_head<1><<<g, 256, 0, st>>>(N.d0.a, wo, bo, N.c, N.H, N.W, tx, ty, N.out); break;
            case 2: k_out_head<2><<<g, 256, 0, st>>>(N.d0.a, wo, bo, N.c, N.H, N.W, tx, ty, N.out); break;
            default: k_out_head<3><<<g, 256, 0, st>>>(N.d0.a, wo, bo, N.c, N.H, N.W, tx, ty, N.out); break;
        }
        FEM_HIP_CHECK(hipGetLastError());
        return 0;
    }
    // with k smoothing passes the 1x1 layer writes where k alternating passes end in N.out
    float *a = (N.out_smooth & 1) ? N.ys : N.out;
    k_out_fwd<<<grid1(P0), 256, 0, st>>>(N.d0.a, N.w + N.out_woff, N.w + N.out_boff, N.c, P0, a);
    for (int k = 0; k < N.out_smooth; ++k) {
        float *b = a == N.out ? N.ys : N.out;
        k_binom<<<grid1(P0), 256, 0, st>>>(a, N.H, N.W, P0, b);
        a = b;
    }
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

int forward(UNet &N, int B, const float *in, hipStream_t st) {
    const int64_t P0 = pixels(N, 0, B);
    k_make_input<<<grid1(P0), 256, 0, st>>>(in, N.x8.a, P0);
    FEM_HIP_CHECK(hipGetLastError());
    return forward_x8(N, B, st);
}

// loss and every parameter gradient (into N.g) for the forward of `in` held in N.out
int backward(UNet &N, int B, const float *in, const float *target, double *loss, hipStream_t st) {
    const int64_t HW = (int64_t)N.H * N.W, P0 = HW * B;
    dim3 lg(N.loss_slices, B);
    // gradient of the (smoothed) output; with smoothing it is passed back
    // through the same passes (their own adjoint), ending in N.gy, before the
    // 1x1 layer's gradients are formed
    const bool sm = N.out_smooth > 0;
    float *ga = (N.out_smooth & 1) ? N.ys : N.gy;
    bf16 *gd0 = sm ? nullptr : N.d0.g;
    if (N.loss_kind == FEM_UNET_LOSS_ENERGY) {
        k_eloss_part<<<lg, 256, 0, st>>>(N.out, target, in, N.H, N.nu_scale, N.loss_slices, N.lpart);
        k_eloss_fin<<<1, 64, 0, st>>>(N.lpart, B, N.loss_slices, N.sums, loss);
        k_eloss_bwd<<<grid1(P0), 256, 0, st>>>(N.out, target, in, N.sums, N.w + N.out_woff, N.c, N.H, B, N.nu_scale,
                                               ga, gd0);
    } else {
        k_loss_part<<<lg, 256, 0, st>>>(N.out, target, HW, N.loss_slices, N.lpart);
        k_loss_fin<<<1, 64, 0, st>>>(N.lpart, B, N.loss_slices, N.sums, loss);
        k_out_bwd<<<grid1(P0), 256, 0, st>>>(N.out, target, N.sums, N.w + N.out_woff, N.c, HW, B, ga, gd0);
    }
    if (sm) {
        for (int k = 0; k < N.out_smooth; ++k) {
            float *gb = ga == N.gy ? N.ys : N.gy;
            k_binom<<<grid1(P0), 256, 0, st>>>(ga, N.H, N.W, P0, gb);
            ga = gb;
        }
        k_out_gd0<<<grid1(P0), 256, 0, st>>>(N.gy, N.w + N.out_woff, N.c, P0, N.d0.g);
    }
    const int64_t so = wgrad_splits(P0);
    if (N.c == 16) k_out_wgrad<16><<<(unsigned)so, 256, 0, st>>>(N.d0.a, N.gy, P0, N.partial);
    else k_out_wgrad<32><<<(unsigned)so, 256, 0, st>>>(N.d0.a, N.gy, P0, N.partial);
    k_sum_splits<<<1, 256, 0, st>>>(N.partial, (int)so, N.c + 1, N.g + N.out_woff);
    FEM_HIP_CHECK(hipGetLastError());
    const auto &L = N.L;
    int rc = 0;
    auto ok = [&](int r) {
        if (!rc) rc = r;
    };
    ok(conv_bwd(N, L[16], N.d0a, nullptr, N.d0, true, B, st));
    ok(conv_bwd(N, L[15], N.u0, &N.e0, N.d0a, true, B, st));
    ok(up_bwd(N, L[14], N.d1, N.u0, B, st));
    ok(conv_bwd(N, L[13], N.d1a, nullptr, N.d1, true, B, st));
    ok(conv_bwd(N, L[12], N.u1, &N.e1, N.d1a, true, B, st));
    ok(up_bwd(N, L[11], N.d2, N.u1, B, st));
    ok(conv_bwd(N, L[10], N.d2a, nullptr, N.d2, true, B, st));
    ok(conv_bwd(N, L[9], N.u2, &N.e2, N.d2a, true, B, st));
    ok(up_bwd(N, L[8], N.mm, N.u2, B, st));
    ok(conv_bwd(N, L[7], N.ma, nullptr, N.mm, true, B, st));
    ok(conv_bwd(N, L[6], N.p2, nullptr, N.ma, true, B, st));
    ok(pool_bwd(N, N.e2, N.p2, B, st));
    ok(conv_bwd(N, L[5], N.e2a, nullptr, N.e2, true, B, st));
    ok(conv_bwd(N, L[4], N.p1, nullptr, N.e2a, true, B, st));
    ok(pool_bwd(N, N.e1, N.p1, B, st));
    ok(conv_bwd(N, L[3], N.e1a, nullptr, N.e1, true, B, st));
    ok(conv_bwd(N, L[2], N.p0, nullptr, N.e1a, true, B, st));
    ok(pool_bwd(N, N.e0, N.p0, B, st));
    ok(conv_bwd(N, L[1], N.e0a, nullptr, N.e0, true, B, st));
    ok(conv_bwd(N, L[0], N.x8, nullptr, N.e0a, false, B, st));
    return rc;
}

void add_layer(UNet &N, int kind, int lvl, int C1, int C2, int Cout) {
    Layer l;
    l.kind = kind;
    l.lvl = lvl;
    l.C1 = C1;
    l.C2 = C2;
    l.Cout = Cout;
    l.woff = N.nparam;
    if (kind == CONV) {
        l.boff = l.woff + (int64_t)9 * l.Cin() * Cout;
        l.KBf = (9 * l.Cin() + 31) / 32;
        l.NTf = Cout / 16;
        l.KBb = (9 * Cout + 31) / 32;
        l.NTb = (l.Cin() + 15) / 16;
    } else {
        l.boff = l.woff + (int64_t)C1 * 4 * Cout;
        l.KBf = (C1 + 31) / 32;
        l.NTf = 4 * Cout / 16;
        l.KBb = (4 * Cout + 31) / 32;
        l.NTb = C1 / 16;
    }
    N.nparam = l.boff + Cout;
    N.L.push_back(l);
}

// He-normal weights (std sqrt(2 / fan_in)), zero biases; the first layer's
// padding input channels 2..7 get zero weights.
void init_params(const UNet &N, uint64_t seed, std::vector<float> &w) {
    std::mt19937_64 gen(seed);
    w.assign((size_t)N.nparam, 0.0f);
    for (size_t li = 0; li < N.L.size(); ++li) {
        const Layer &l = N.L[li];
        const int fan_in = l.kind == CONV ? 9 * (li == 0 ? 2 : l.Cin()) : l.C1;
        std::normal_distribution<double> nd(0.0, std::sqrt(2.0 / fan_in));
        const int64_t nw = l.boff - l.woff;
        for (int64_t i = 0; i < nw; ++i) {
            double v = nd(gen);
            if (li == 0 && (i / l.Cout) % l.Cin() >= 2) v = 0.0;
            w[(size_t)(l.woff + i)] = (float)v;
        }
    }
    std::normal_distribution<double> nd(0.0, std::sqrt(1.0 / N.c));
    for (int ci = 0; ci < N.c; ++ci) w[(size_t)(N.out_woff + ci)] = (float)nd(gen);
}

}  // namespace

}  // namespace fem

struct fem_unet {
    fem::UNet net;
};

namespace {

using fem::set_error;

hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

int check_net(const fem_unet *n) { return n ? FEM_OK : set_error(FEM_EINVAL, "network is NULL"); }

int check_batch(const fem_unet *n, int B) {
    if (B < 1 || B > n->net.maxB) return set_error(FEM_EINVAL, "batch must be in [1, max_batch]");
    return FEM_OK;
}

}  // namespace

namespace fem {

int unet_grid_precondition(fem_unet *net, int grid_n, const double *r, double cval, const uint8_t *mask, double *z,
                           hipStream_t st) {
    UNet &N = net->net;
    if (grid_n != N.H || grid_n != N.W) return set_error(FEM_EINVAL, "grid size must equal the network image size");
    const int64_t n_int = (int64_t)(grid_n - 1) * (grid_n - 1);
    const int parts = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n_int + 255) / 256));
    k_interior_sumsq<<<parts, 256, 0, st>>>(r, grid_n, N.gpart);
    k_grid_scale<<<1, 256, 0, st>>>(N.gpart, parts, grid_n, N.gpart + kGridScale);
    k_grid_in8<<<grid1((int64_t)grid_n * grid_n), 256, 0, st>>>(r, N.gpart + kGridScale, grid_n, (float)cval,
                                                                 N.x8.a);
    FEM_HIP_CHECK(hipGetLastError());
    if (int rc = forward_x8(N, 1, st)) return rc;
    k_grid_out<<<grid1((int64_t)(grid_n + 1) * (grid_n + 1)), 256, 0, st>>>(N.out, grid_n, mask, z);
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

int unet_grid_pair(fem_unet *net, int grid_n, const double *r, const double *u, const double *x, double cval,
                   float *in2, float *tgt, hipStream_t st) {
    UNet &N = net->net;
    if (grid_n != N.H || grid_n != N.W) return set_error(FEM_EINVAL, "grid size must equal the network image size");
    const int64_t n_int = (int64_t)(grid_n - 1) * (grid_n - 1);
    const int parts = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n_int + 255) / 256));
    const int g = grid1((int64_t)grid_n * grid_n);
    k_interior_sumsq<<<parts, 256, 0, st>>>(r, grid_n, N.gpart);
    k_grid_scale<<<1, 256, 0, st>>>(N.gpart, parts, grid_n, N.gpart + kGridScale);
    k_grid_in<<<g, 256, 0, st>>>(r, N.gpart + kGridScale, grid_n, (float)cval, in2);
    k_interior_sumsq_diff<<<parts, 256, 0, st>>>(u, x, grid_n, N.gpart + 1024);
    k_grid_scale<<<1, 256, 0, st>>>(N.gpart + 1024, parts, grid_n, N.gpart + kGridScale + 1);
    k_grid_target<<<g, 256, 0, st>>>(u, x, N.gpart + kGridScale + 1, grid_n, tgt);
    FEM_HIP_CHECK(hipGetLastError());
    return 0;
}

}  // namespace fem

extern "C" {

int fem_unet_create(int H, int W, int max_batch, int channels, uint64_t seed, void *stream, fem_unet **out) {
    fem::last_error().clear();
    if (!out) return set_error(FEM_EINVAL, "out is NULL");
    *out = nullptr;
    if (H < 8 || W < 8 || H % 8 || W % 8 || H > 8192 || W > 8192)
        return set_error(FEM_EINVAL, "H and W must be multiples of 8 in [8, 8192]");
    if (channels != 16 && channels != 32) return set_error(FEM_EINVAL, "channels must be 16 or 32");
    if (max_batch < 1 || (int64_t)max_batch * H * W > ((int64_t)1 << 27))
        return set_error(FEM_EINVAL, "max_batch * H * W must be in [1, 2^27]");
    fem_unet *net = new (std::nothrow) fem_unet();
    if (!net) return set_error(FEM_ENOMEM, "host allocation failed");
    fem::UNet &N = net->net;
    N.H = H;
    N.W = W;
    N.maxB = max_batch;
    N.c = channels;
    const int c = channels;
    using fem::CONV;
    using fem::UP;
    fem::add_layer(N, CONV, 0, 8, 0, c);
    fem::add_layer(N, CONV, 0, c, 0, c);
    fem::add_layer(N, CONV, 1, c, 0, 2 * c);
    fem::add_layer(N, CONV, 1, 2 * c, 0, 2 * c);
    fem::add_layer(N, CONV, 2, 2 * c, 0, 4 * c);
    fem::add_layer(N, CONV, 2, 4 * c, 0, 4 * c);
    fem::add_layer(N, CONV, 3, 4 * c, 0, 8 * c);
    fem::add_layer(N, CONV, 3, 8 * c, 0, 8 * c);
    fem::add_layer(N, UP, 3, 8 * c, 0, 4 * c);
    fem::add_layer(N, CONV, 2, 4 * c, 4 * c, 4 * c);
    fem::add_layer(N, CONV, 2, 4 * c, 0, 4 * c);
    fem::add_layer(N, UP, 2, 4 * c, 0, 2 * c);
    fem::add_layer(N, CONV, 1, 2 * c, 2 * c, 2 * c);
    fem::add_layer(N, CONV, 1, 2 * c, 0, 2 * c);
    fem::add_layer(N, UP, 1, 2 * c, 0, c);
    fem::add_layer(N, CONV, 0, c, c, c);
    fem::add_layer(N, CONV, 0, c, 0, c);
    N.out_woff = N.nparam;
    N.out_boff = N.out_woff + c;
    N.nparam = N.out_boff + 1;

    // one device arena: parameters, Adam state, packed operands, activations, scratch
    struct Item {
        void **ptr;
        size_t bytes;
    };
    std::vector<Item> items;
    auto add = [&](void **p, size_t bytes) { items.push_back({p, bytes}); };
    const int64_t np = N.nparam;
    add((void **)&N.w, np * 4);
    add((void **)&N.g, np * 4);
    add((void **)&N.m, np * 4);
    add((void **)&N.v, np * 4);
    for (size_t li = 0; li < N.L.size(); ++li) {
        fem::Layer &l = N.L[li];
        add((void **)&l.Bf, (size_t)l.KBf * l.NTf * 512 * 2);
        if (li != 0) add((void **)&l.Bb, (size_t)l.KBb * l.NTb * 512 * 2);
    }
    const int B = max_batch;
    auto tens = [&](fem::Tensor &t, int lvl, int C) {
        t.lvl = lvl;
        t.C = C;
        const size_t bytes = (size_t)fem::pixels(N, lvl, B) * C * 2;
        add((void **)&t.a, bytes);
        add((void **)&t.g, bytes);
    };
    tens(N.x8, 0, 8);
    tens(N.e0a, 0, c);
    tens(N.e0, 0, c);
    tens(N.p0, 1, c);
    tens(N.e1a, 1, 2 * c);
    tens(N.e1, 1, 2 * c);
    tens(N.p1, 2, 2 * c);
    tens(N.e2a, 2, 4 * c);
    tens(N.e2, 2, 4 * c);
    tens(N.p2, 3, 4 * c);
    tens(N.ma, 3, 8 * c);
    tens(N.mm, 3, 8 * c);
    tens(N.u2, 2, 4 * c);
    tens(N.d2a, 2, 4 * c);
    tens(N.d2, 2, 4 * c);
    tens(N.u1, 1, 2 * c);
    tens(N.d1a, 1, 2 * c);
    tens(N.d1, 1, 2 * c);
    tens(N.u0, 0, c);
    tens(N.d0a, 0, c);
    tens(N.d0, 0, c);
    const int64_t P0 = fem::pixels(N, 0, B);
    add((void **)&N.out, P0 * 4);
    add((void **)&N.gy, P0 * 4);
    add((void **)&N.ys, P0 * 4);
    int64_t cap = fem::wgrad_splits(P0) * (c + 1);
    for (const auto &l : N.L) {
        const int64_t M = fem::pixels(N, l.lvl, B);
        const int R1 = l.kind == CONV ? 9 * l.Cin() + 1 : l.C1 + 1;
        const int64_t need = l.kind == CONV ? (int64_t)R1 * l.Cout : (int64_t)R1 * 4 * l.Cout;
        const int rpb = l.kind == CONV ? fem::conv_wgrad_rows(l.Cout / 16) : 64;
        // the row GEMM fallback of a convolution uses 64-row blocks: the larger of the two counts
        cap = std::max(cap, fem::wgrad_splits(M, fem::wgrad_slice(M, R1, rpb)) * need);
        cap = std::max(cap, fem::wgrad_splits(M, fem::wgrad_slice(M, R1)) * need);
    }
    N.partial_cap = cap;
    add((void **)&N.partial, cap * 4);
    add((void **)&N.sums, (size_t)3 * B * 8);
    add((void **)&N.lpart, (size_t)3 * B * N.loss_slices * 8);
    add((void **)&N.gpart, (fem::kGridScale + 8) * 8);
    size_t total = 0;
    std::vector<size_t> offs;
    for (auto &it : items) {
        offs.push_back(total);
        total += (it.bytes + 255) / 256 * 256;
    }
    if (hipMalloc(&N.arena, total) != hipSuccess) {
        (void)hipGetLastError();
        delete net;
        return set_error(FEM_ENOMEM, "device allocation of the network failed");
    }
    for (size_t i = 0; i < items.size(); ++i) *items[i].ptr = static_cast<char *>(N.arena) + offs[i];
    hipStream_t st = S(stream);
    std::vector<float> w0;
    fem::init_params(N, seed, w0);
    int rc = 0;
    if (hipMemsetAsync(N.arena, 0, total, st) != hipSuccess ||
        hipMemcpyAsync(N.w, w0.data(), np * 4, hipMemcpyHostToDevice, st) != hipSuccess)
        rc = set_error(FEM_EHIP, "upload of the initial parameters failed");
    if (!rc) rc = fem::repack(N, st);
    if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = set_error(FEM_EHIP, "stream synchronisation failed");
    if (rc) {
        (void)hipFree(N.arena);
        delete net;
        return rc;
    }
    *out = net;
    return FEM_OK;
}

int fem_unet_destroy(fem_unet *net) {
    if (!net) return FEM_OK;
    int rc = FEM_OK;
    if (net->net.arena && hipFree(net->net.arena) != hipSuccess) rc = set_error(FEM_EHIP, "hipFree failed");
    delete net;
    return rc;
}

int fem_unet_param_count(const fem_unet *net, int64_t *count) {
    if (int rc = check_net(net)) return rc;
    if (!count) return set_error(FEM_EINVAL, "count is NULL");
    *count = net->net.nparam;
    return FEM_OK;
}

int fem_unet_get_params(const fem_unet *net, float *d_params, void *stream) {
    if (int rc = check_net(net)) return rc;
    if (!d_params) return set_error(FEM_EINVAL, "params is NULL");
    FEM_HIP_CHECK(hipMemcpyAsync(d_params, net->net.w, net->net.nparam * 4, hipMemcpyDeviceToDevice, S(stream)));
    return FEM_OK;
}

int fem_unet_set_params(fem_unet *net, const float *d_params, void *stream) {
    if (int rc = check_net(net)) return rc;
    if (!d_params) return set_error(FEM_EINVAL, "params is NULL");
    fem::UNet &N = net->net;
    hipStream_t st = S(stream);
    FEM_HIP_CHECK(hipMemcpyAsync(N.w, d_params, N.nparam * 4, hipMemcpyDeviceToDevice, st));
    FEM_HIP_CHECK(hipMemsetAsync(N.m, 0, N.nparam * 4, st));
    FEM_HIP_CHECK(hipMemsetAsync(N.v, 0, N.nparam * 4, st));
    N.step = 0;
    return fem::repack(N, st);
}

int fem_unet_forward(fem_unet *net, int batch, const float *d_in, float *d_out, void *stream) {
    if (int rc = check_net(net)) return rc;
    if (int rc = check_batch(net, batch)) return rc;
    if (!d_in || !d_out) return set_error(FEM_EINVAL, "NULL argument");
    fem::UNet &N = net->net;
    hipStream_t st = S(stream);
    if (int rc = fem::forward(N, batch, d_in, st)) return rc;
    FEM_HIP_CHECK(hipMemcpyAsync(d_out, N.out, fem::pixels(N, 0, batch) * 4, hipMemcpyDeviceToDevice, st));
    return FEM_OK;
}

int fem_unet_loss_grad(fem_unet *net, int batch, const float *d_in, const float *d_target, double *d_loss,
                       float *d_grad, void *stream) {
    if (int rc = check_net(net)) return rc;
    if (int rc = check_batch(net, batch)) return rc;
    if (!d_in || !d_target || !d_loss) return set_error(FEM_EINVAL, "NULL argument");
    fem::UNet &N = net->net;
    hipStream_t st = S(stream);
    if (int rc = fem::forward(N, batch, d_in, st)) return rc;
    if (int rc = fem::backward(N, batch, d_in, d_target, d_loss, st)) return rc;
    if (d_grad) FEM_HIP_CHECK(hipMemcpyAsync(d_grad, N.g, N.nparam * 4, hipMemcpyDeviceToDevice, st));
    return FEM_OK;
}

int fem_unet_set_loss(fem_unet *net, int kind, double nu_scale) {
    if (int rc = check_net(net)) return rc;
    fem::UNet &N = net->net;
    if (kind == FEM_UNET_LOSS_L2) {
        N.loss_kind = kind;
        N.nu_scale = 0.0;
        return FEM_OK;
    }
    if (kind != FEM_UNET_LOSS_ENERGY) return set_error(FEM_EINVAL, "unknown loss kind");
    if (N.H != N.W) return set_error(FEM_EINVAL, "the energy loss needs square images");
    if (!(nu_scale >= 0.0) || !std::isfinite(nu_scale)) return set_error(FEM_EINVAL, "nu_scale must be finite and >= 0");
    N.loss_kind = kind;
    N.nu_scale = nu_scale;
    return FEM_OK;
}

int fem_unet_set_output_smoothing(fem_unet *net, int passes) {
    if (int rc = check_net(net)) return rc;
    if (passes < 0 || passes > 8) return set_error(FEM_EINVAL, "output smoothing passes must be in [0, 8]");
    net->net.out_smooth = passes;
    return FEM_OK;
}

int fem_unet_train_step(fem_unet *net, int batch, const float *d_in, const float *d_target, float lr,
                        double *d_loss, void *stream) {
    if (int rc = check_net(net)) return rc;
    if (int rc = check_batch(net, batch)) return rc;
    if (!d_in || !d_target) return set_error(FEM_EINVAL, "NULL argument");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return set_error(FEM_EINVAL, "lr must be finite and > 0");
    fem::UNet &N = net->net;
    hipStream_t st = S(stream);
    if (int rc = fem::forward(N, batch, d_in, st)) return rc;
    if (int rc = fem::backward(N, batch, d_in, d_target, d_loss, st)) return rc;
    N.step += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 - std::pow(b1, (double)N.step)), c2 = (float)(1.0 - std::pow(b2, (double)N.step));
    fem::k_adam<<<fem::grid1(N.nparam), 256, 0, st>>>(N.w, N.g, N.m, N.v, N.nparam, lr, (float)b1, (float)b2, 1e-8f,
                                                      c1, c2);
    FEM_HIP_CHECK(hipGetLastError());
    return fem::repack(N, st);
}

int fem_unet_precondition(fem_unet *net, int grid_n, const double *d_r, double cval, const uint8_t *d_mask,
                          double *d_z, void *stream) {
    if (int rc = check_net(net)) return rc;
    if (!d_r || !d_z) return set_error(FEM_EINVAL, "NULL argument");
    if (d_r == d_z) return set_error(FEM_EINVAL, "z must not alias r");
    if (!std::isfinite(cval)) return set_error(FEM_EINVAL, "cval must be finite");
    return fem::unet_grid_precondition(net, grid_n, d_r, cval, d_mask, d_z, S(stream));
}

int fem_unet_make_pair(fem_unet *net, int grid_n, const double *d_r, const double *d_u, const double *d_x,
                       double cval, float *d_in, float *d_target, void *stream) {
    if (int rc = check_net(net)) return rc;
    if (!d_r || !d_u || !d_x || !d_in || !d_target) return set_error(FEM_EINVAL, "NULL argument");
    if (!std::isfinite(cval)) return set_error(FEM_EINVAL, "cval must be finite");
    return fem::unet_grid_pair(net, grid_n, d_r, d_u, d_x, cval, d_in, d_target, S(stream));
}

}  // extern "C"
