// learned.hip -- a message-passing network that predicts a sparse approximate inverse
// (learned preconditioner for the refinement's inner CG), with hand-written forward,
// backward and Adam kernels.  Not part of the paper's method (the paper lists
// mixed-precision preconditioned Krylov methods as future work, Sec. 5).
//
// For a Stieltjes matrix A (SPD, non-positive off-diagonal entries, like every diffusion
// matrix) with a symmetric pattern (hi = leading DD component):
//   minv_i = 1/hi(a_ii);  w_ij = -hi(a_ij)/sqrt(hi(a_ii) hi(a_jj))           (float)
//   f_i = [sum_j w_ij, sum_j w_ij^2, deg_i/8, 1]
//   h0 = relu(f W0 + b0);  l = 1..3: m_i = sum_j w_ij h_j,  h = relu(h Ws + m Wn + b)
//   u_i = h_i.wu + bu;  v_ij = sum_k qv_k (h_ik h_jk) + bv                   (v_ij = v_ji)
//   g_ij = tanh(v_ij)^2 in [0, 1);  c_ij = g_ij w_ij;  delta_i = log(1 + u_i^2) >= 0
//   M_ii = (1 + delta_i) minv_i;  M_ij = c_ij sqrt(minv_i minv_j)
// i.e. M = S (I + Delta + G o W) S with S = D^-1/2, a damped first-order Neumann
// approximation of A^-1 = S (I - W)^-1 S.  M is SPD: W >= 0 entrywise with spectral
// radius below 1 (I - W = S A S is SPD), so rho(G o W) <= rho(W) < 1 and I + Delta +
// G o W is positive definite.  With zero weights M is exactly the Jacobi inverse
// diagonal.  Training loss of a pair (r, e = A^-1 r):
//   L = (M r - e)^T A (M r - e) / e^T A e.
// Weights are bfloat16 values (the float32 master copy is rounded to nearest-even on
// every use); dense-layer inputs are rounded to bfloat16 too and products accumulate in
// float32 (a bf16 x bf16 product is exact in float32).  The backward pass treats the
// bf16 roundings as the identity.  Every reduction has a fixed order (CSR row order,
// fixed node/edge blocks summed in block order), so results are deterministic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "common.hpp"

namespace mpk {

constexpr int kH = 64;        // hidden width
constexpr int kF = 4;         // node features
constexpr int kNodeBlock = 256;   // nodes per partial-gradient block
constexpr int kEdgeBlock = 1024;  // edges per partial-gradient block

// parameter offsets (float32 master vector)
constexpr int OFF_W0 = 0;
constexpr int OFF_B0 = OFF_W0 + kF * kH;
constexpr int OFF_L1 = OFF_B0 + kH;                 // layer l: Ws, Wn, b
constexpr int LAYER_SZ = kH * kH * 2 + kH;
constexpr int OFF_WU = OFF_L1 + 3 * LAYER_SZ;
constexpr int OFF_BU = OFF_WU + kH;
constexpr int OFF_QV = OFF_BU + 1;
constexpr int OFF_BV = OFF_QV + kH;
constexpr int N_PARAMS = OFF_BV + 1;

inline int off_ws(int l) { return OFF_L1 + (l - 1) * LAYER_SZ; }
inline int off_wn(int l) { return off_ws(l) + kH * kH; }
inline int off_b(int l) { return off_wn(l) + kH * kH; }

__device__ __forceinline__ float bfr(float x)
{
    uint32_t u = __float_as_uint(x);
    const uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7FFFu + lsb) & 0xFFFF0000u;
    return __uint_as_float(u);
}

__device__ __forceinline__ float softplusf(float x) { return x > 20.f ? x : log1pf(expf(x)); }

}  // namespace mpk

struct mp_mpnn {
    float *d_theta = nullptr;   // master parameters
    float *d_grad = nullptr;    // accumulated gradients
    float *d_m = nullptr;       // Adam first moment
    float *d_v = nullptr;       // Adam second moment
};

struct mp_graph {
    int32_t n = 0;
    int64_t nnz = 0;
    const int32_t *row_ptr = nullptr;   // caller's pattern (device)
    const int32_t *col_idx = nullptr;
    const double *a = nullptr;           // caller's DD values (device)
    int32_t *d_rows = nullptr;           // row of each element
    int32_t *d_rev = nullptr;            // position of (j, i) for element (i, j)
    float *d_w = nullptr;                // edge weights (0 on the diagonal)
    float *d_f = nullptr;                // node features n x 4
    double *d_minv = nullptr;            // 1 / hi(a_ii)
    float *d_H[4] = {nullptr, nullptr, nullptr, nullptr};   // activations n x 64
    float *d_Mg[4] = {nullptr, nullptr, nullptr, nullptr};  // aggregated messages (layers 1..3)
    float *d_u = nullptr, *d_v = nullptr, *d_c = nullptr;   // readouts, c_ij
    float *d_du = nullptr, *d_dv = nullptr;                 // their gradients (summed over pairs)
    float *d_dH = nullptr, *d_dH2 = nullptr, *d_dMg = nullptr;
    float *d_wpart = nullptr;            // partial weight gradients (blocks x 64 x 64)
    double *d_vec = nullptr;             // 5 x n doubles of scratch for the loss
    double *d_dpart = nullptr;           // dot partials
    double *d_M = nullptr;               // assembled M values (nnz)
    int32_t *d_bad = nullptr;            // set-up check result (1 value)
    void *d_arena = nullptr;             // one device allocation holding every buffer above
    int32_t nblk = 0, eblk = 0;
};

namespace mpk {

// ---------------------------------------------------------------------------
// graph set-up
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_g_diag(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                const double *__restrict__ a, double *__restrict__ minv,
                                                int32_t *__restrict__ rows, int32_t *__restrict__ bad)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double d = 0.0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            rows[k] = (int32_t)i;
            if (ci[k] == i) d = a[k];
        }
        if (!(d > 0.0)) atomicMin(bad, (int32_t)i);
        minv[i] = 1.0 / d;
    }
}

__global__ __launch_bounds__(256) void k_g_edges(int32_t n, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci, const double *__restrict__ a,
                                                 const double *__restrict__ minv, float *__restrict__ w,
                                                 float *__restrict__ f, int32_t *__restrict__ rev,
                                                 int32_t *__restrict__ bad)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double s1 = 0.0, s2 = 0.0;
        int deg = 0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int32_t j = ci[k];
            float wk = 0.f;
            if (j != i) {
                // 1/sqrt(a_ii a_jj) = sqrt(minv_i minv_j); a positive off-diagonal entry
                // (not a Stieltjes matrix) is refused
                if (a[k] > 0.0) atomicMin(bad, (int32_t)i);
                wk = (float)(-a[k] * sqrt(minv[i] * minv[j]));
                ++deg;
                // reverse element (j, i): columns of row j are sorted
                int32_t lo = rp[j], hi = rp[j + 1] - 1, pos = -1;
                while (lo <= hi) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (ci[mid] == i) {
                        pos = mid;
                        break;
                    }
                    if (ci[mid] < i) lo = mid + 1;
                    else hi = mid - 1;
                }
                if (pos < 0) atomicMin(bad, (int32_t)i);
                rev[k] = pos < 0 ? k : pos;
            } else {
                rev[k] = k;
            }
            w[k] = wk;
            s1 += (double)wk;
            s2 += (double)wk * (double)wk;
        }
        f[i * 4 + 0] = (float)s1;
        f[i * 4 + 1] = (float)s2;
        f[i * 4 + 2] = (float)deg / 8.0f;
        f[i * 4 + 3] = 1.0f;
    }
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------

// H = relu(bf(X1) bf(W1) + bf(X2) bf(W2) + b); thread per (node, output), 4 nodes per block
template <int K1, bool X2>
__global__ __launch_bounds__(256) void k_dense(int32_t n, const float *__restrict__ X1, const float *__restrict__ W1,
                                               const float *__restrict__ X2p, const float *__restrict__ W2,
                                               const float *__restrict__ b, float *__restrict__ H)
{
    __shared__ float sW1[K1 * kH];
    __shared__ float sW2[X2 ? kH * kH : 1];
    __shared__ float sx1[4][K1];
    __shared__ float sx2[4][X2 ? kH : 1];
    const int t = threadIdx.x;
    for (int i = t; i < K1 * kH; i += 256) sW1[i] = bfr(W1[i]);
    if constexpr (X2)
        for (int i = t; i < kH * kH; i += 256) sW2[i] = bfr(W2[i]);
    const int local = t >> 6, o = t & 63;
    const int64_t node = (int64_t)blockIdx.x * 4 + local;
    if (node < n) {
        if (o < K1) sx1[local][o] = bfr(X1[node * K1 + o]);
        if constexpr (X2) sx2[local][o] = bfr(X2p[node * kH + o]);
    }
    __syncthreads();
    if (node >= n) return;
    float acc = 0.f;
#pragma unroll 8
    for (int k = 0; k < K1; ++k) acc = fmaf(sx1[local][k], sW1[k * kH + o], acc);
    if constexpr (X2) {
#pragma unroll 8
        for (int k = 0; k < kH; ++k) acc = fmaf(sx2[local][k], sW2[k * kH + o], acc);
    }
    acc = acc + b[o];
    H[node * kH + o] = acc > 0.f ? acc : 0.f;
}

// ---------------------------------------------------------------------------
// hidden dense layers on the matrix cores (bf16 operands, fp32 accumulation)
// ---------------------------------------------------------------------------

typedef short v4bf __attribute__((ext_vector_type(4)));   // four bfloat16 bit patterns
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_bits(float x) { return (short)(__float_as_uint(bfr(x)) >> 16); }

// One wavefront computes a 16-node x 64-output block as 4 column blocks of the
// 16x16x16 bf16 MFMA.  Operand layout of that instruction (lane l, element v):
// A[i][k] with i = l % 16, k = 4 (l / 16) + v; B[k][j] with k = 4 (l / 16) + v,
// j = l % 16; D[i][j] with i = 4 (l / 16) + v, j = l % 16.
//   out = X1 W1 + X2 W2 (64 inputs each), W given in LDS as bf16 [k][o] (or, with
//   TRANS, as [o][k] so that the product is X W^T)
// SPLIT: X is not a bfloat16 quantity (a gradient); it is split exactly enough as
// hi + lo with hi = bf(X), lo = bf(X - hi) and both parts are multiplied (about 16
// significant bits, far below the float32 accumulation's own error budget here).
template <bool TRANS, bool SPLIT>
__device__ __forceinline__ void mfma_rows16(const float *__restrict__ X, int64_t node0, int32_t n,
                                            const short *__restrict__ sW, v4f (&acc)[4], bool relu_mask,
                                            const float *__restrict__ Hmask)
{
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    const int64_t node = node0 + r;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        v4bf a, alo;
        const int k0 = 16 * kb + 4 * g;
        if (node < n) {
            const float4 xv = *reinterpret_cast<const float4 *>(X + node * kH + k0);
            float x4[4] = {xv.x, xv.y, xv.z, xv.w};
            if (relu_mask) {
                const float4 hv = *reinterpret_cast<const float4 *>(Hmask + node * kH + k0);
                x4[0] = hv.x > 0.f ? x4[0] : 0.f;
                x4[1] = hv.y > 0.f ? x4[1] : 0.f;
                x4[2] = hv.z > 0.f ? x4[2] : 0.f;
                x4[3] = hv.w > 0.f ? x4[3] : 0.f;
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                a[v] = bf16_bits(x4[v]);
                if constexpr (SPLIT) alo[v] = bf16_bits(x4[v] - bfr(x4[v]));
            }
        } else {
            a = v4bf{0, 0, 0, 0};
            alo = a;
        }
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            v4bf bm;
            const int o = 16 * cb + r;
#pragma unroll
            for (int v = 0; v < 4; ++v) bm[v] = TRANS ? sW[o * kH + k0 + v] : sW[(k0 + v) * kH + o];
            acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bm, acc[cb], 0, 0, 0);
            if constexpr (SPLIT) acc[cb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, bm, acc[cb], 0, 0, 0);
        }
    }
}

// H = relu(bf(X1) bf(W1) + bf(X2) bf(W2) + b) for the hidden layers; 64 nodes per block
__global__ __launch_bounds__(256) void k_dense_mfma(int32_t n, const float *__restrict__ X1,
                                                    const float *__restrict__ W1, const float *__restrict__ X2,
                                                    const float *__restrict__ W2, const float *__restrict__ b,
                                                    float *__restrict__ H)
{
    __shared__ short sW[2][kH * kH];
    const int t = threadIdx.x;
    for (int i = t; i < kH * kH; i += 256) {
        sW[0][i] = bf16_bits(W1[i]);
        sW[1][i] = bf16_bits(W2[i]);
    }
    __syncthreads();
    const int64_t node0 = (int64_t)blockIdx.x * 64 + (t >> 6) * 16;
    v4f acc[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) acc[cb] = v4f{0.f, 0.f, 0.f, 0.f};
    mfma_rows16<false, false>(X1, node0, n, sW[0], acc, false, nullptr);
    mfma_rows16<false, false>(X2, node0, n, sW[1], acc, false, nullptr);
    const int lane = t & 63;
    const int r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int o = 16 * cb + r;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t node = node0 + 4 * g + v;
            if (node < n) {
                const float z = acc[cb][v] + b[o];
                H[node * kH + o] = z > 0.f ? z : 0.f;
            }
        }
    }
}

// dX1 = dZ bf(W1)^T, dX2 = dZ bf(W2)^T with dZ = dH o [Hout > 0] (split in two bf16
// parts); 64 nodes per block
__global__ __launch_bounds__(256) void k_dense_bwd_x_mfma(int32_t n, const float *__restrict__ dH,
                                                          const float *__restrict__ Hout,
                                                          const float *__restrict__ W1, float *__restrict__ dX1,
                                                          const float *__restrict__ W2, float *__restrict__ dX2)
{
    __shared__ short sW[2][kH * kH];
    const int t = threadIdx.x;
    for (int i = t; i < kH * kH; i += 256) {
        sW[0][i] = bf16_bits(W1[i]);
        sW[1][i] = bf16_bits(W2[i]);
    }
    __syncthreads();
    const int64_t node0 = (int64_t)blockIdx.x * 64 + (t >> 6) * 16;
    const int lane = t & 63;
    const int r = lane & 15, g = lane >> 4;
    for (int w = 0; w < 2; ++w) {
        v4f acc[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = v4f{0.f, 0.f, 0.f, 0.f};
        mfma_rows16<true, true>(dH, node0, n, sW[w], acc, true, Hout);
        float *out = w ? dX2 : dX1;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int k = 16 * cb + r;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t node = node0 + 4 * g + v;
                if (node < n) out[node * kH + k] = acc[cb][v];
            }
        }
    }
}

// Out_i = base_i + sum_j w_ij X_j (row order); thread per (node, feature)
__global__ __launch_bounds__(256) void k_aggregate(int32_t n, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci, const float *__restrict__ w,
                                                   const float *__restrict__ X, const float *__restrict__ base,
                                                   float *__restrict__ Out)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t node = g >> 6;
    const int f = (int)(g & 63);
    if (node >= n) return;
    float acc = 0.f;
    for (int32_t k = rp[node]; k < rp[node + 1]; ++k) acc = fmaf(w[k], X[(int64_t)ci[k] * kH + f], acc);
    Out[node * kH + f] = base ? base[node * kH + f] + acc : acc;
}

// u_i = bf(h_i).bf(wu) + bu  and, per element, v_ij = sum_k bf(qv_k) (bf(h_ik) bf(h_jk)) + bv
__global__ __launch_bounds__(256) void k_readout(int32_t n, int64_t nnz, const int32_t *__restrict__ rows,
                                                 const int32_t *__restrict__ ci, const float *__restrict__ H,
                                                 const float *__restrict__ theta, float *__restrict__ u,
                                                 float *__restrict__ v)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (int64_t i = g; i < n; i += (int64_t)gridDim.x * 256) {
        float acc = 0.f;
        for (int k = 0; k < kH; ++k) acc = fmaf(bfr(H[i * kH + k]), bfr(theta[OFF_WU + k]), acc);
        u[i] = acc + theta[OFF_BU];
    }
    for (int64_t e = g; e < nnz; e += (int64_t)gridDim.x * 256) {
        const int64_t i = rows[e], j = ci[e];
        float acc = 0.f;
        if (i != j) {
            for (int k = 0; k < kH; ++k) {
                const float p = bfr(H[i * kH + k]) * bfr(H[j * kH + k]);
                acc = fmaf(bfr(theta[OFF_QV + k]), p, acc);
            }
        }
        v[e] = acc + theta[OFF_BV];
    }
}

// c_ij = tanh(v_ij)^2 w_ij, the diagonal and M (float64) on the pattern; one thread per row
__global__ __launch_bounds__(256) void k_assemble(int32_t n, const int32_t *__restrict__ rp,
                                                  const int32_t *__restrict__ ci, const float *__restrict__ u,
                                                  const float *__restrict__ v, const float *__restrict__ w,
                                                  const double *__restrict__ minv, float *__restrict__ c,
                                                  double *__restrict__ M)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        int32_t kd = -1;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int32_t j = ci[k];
            if (j == i) {
                kd = k;
                c[k] = 0.f;
                continue;
            }
            const float th = tanhf(v[k]);
            const float ck = th * th * w[k];
            c[k] = ck;
            M[k] = (double)ck * sqrt(minv[i] * minv[j]);
        }
        const float diag = 1.f + log1pf(u[i] * u[i]);
        if (kd >= 0) M[kd] = (double)diag * minv[i];
    }
}

// ---------------------------------------------------------------------------
// loss (float64) and its gradient with respect to u and v
// ---------------------------------------------------------------------------

// y = V x, each row summed sequentially (binary64)
__global__ __launch_bounds__(256) void k_spmv64(int32_t n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                const double *__restrict__ V, const double *__restrict__ x,
                                                const double *__restrict__ sub, double *__restrict__ y)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double s = 0.0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const double p = V[k] * x[ci[k]];
            s = (k == rp[i]) ? p : s + p;
        }
        y[i] = sub ? s - sub[i] : s;
    }
}

// chunk partials of x.y (lanes then fold), one block per 4096 elements
__global__ __launch_bounds__(256) void k_dot64(int32_t n, const double *__restrict__ x, const double *__restrict__ y,
                                               double *__restrict__ part)
{
    __shared__ double lds[256];
    const int64_t base = (int64_t)blockIdx.x * 4096;
    const int t = threadIdx.x;
    double acc = 0.0;
    for (int64_t k = base + t; k < n && k < base + 4096; k += 256) acc = acc + x[k] * y[k];
    lds[t] = acc;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if (t < off) lds[t] = lds[t] + lds[t + off];
        __syncthreads();
    }
    if (t == 0) part[blockIdx.x] = lds[0];
}

// loss = (d.Ad)/(e.Ae) written to out[0]; out[1] = 2/(e.Ae)
__global__ __launch_bounds__(256) void k_loss_final(const double *__restrict__ pdd, const double *__restrict__ pee, int m,
                                                    double *__restrict__ out)
{
    if (threadIdx.x != 0) return;
    double dd = 0.0, ee = 0.0;
    for (int i = 0; i < m; ++i) {
        dd = dd + pdd[i];
        ee = ee + pee[i];
    }
    out[0] = dd / ee;
    out[1] = 2.0 / ee;
}

// gy = scale * Ad; du_i += G_i 2 u_i / (1 + u_i^2) with G_i = gy_i r_i minv_i;
// dv_k += dc_k w_k 2 tanh(v_k) (1 - tanh^2 v_k) with dc_k = gy_i r_j sqrt(minv_i minv_j)
__global__ __launch_bounds__(256) void k_assemble_bwd(int32_t n, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci, const double *__restrict__ Ad,
                                                      const double *__restrict__ scale, const double *__restrict__ r,
                                                      const double *__restrict__ minv, const float *__restrict__ u,
                                                      const float *__restrict__ v, const float *__restrict__ w,
                                                      float *__restrict__ du, float *__restrict__ dv)
{
    const double sc = scale[1];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double gi = sc * Ad[i];
        const double G = gi * r[i] * minv[i];
        const double ui = (double)u[i];
        du[i] += (float)(G * 2.0 * ui / (1.0 + ui * ui));
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
            const int32_t j = ci[k];
            if (j == i) continue;
            const double dc = gi * r[j] * sqrt(minv[i] * minv[j]);
            const double th = tanh((double)v[k]);
            dv[k] += (float)(dc * (double)w[k] * 2.0 * th * (1.0 - th * th));
        }
    }
}

// ---------------------------------------------------------------------------
// backward through the network
// ---------------------------------------------------------------------------

// dH_i = du_i bf(wu) + sum_{k in row i} (dv_k + dv_rev(k)) bf(qv) bf(h_j); thread per (node, feature)
__global__ __launch_bounds__(256) void k_readout_bwd(int32_t n, const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci, const int32_t *__restrict__ rev,
                                                     const float *__restrict__ H, const float *__restrict__ theta,
                                                     const float *__restrict__ du, const float *__restrict__ dv,
                                                     float *__restrict__ dH)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t node = g >> 6;
    const int f = (int)(g & 63);
    if (node >= n) return;
    const float q = bfr(theta[OFF_QV + f]);
    float acc = du[node] * bfr(theta[OFF_WU + f]);
    for (int32_t k = rp[node]; k < rp[node + 1]; ++k) {
        const int32_t j = ci[k];
        if (j == node) continue;
        acc = fmaf(dv[k] + dv[rev[k]], q * bfr(H[(int64_t)j * kH + f]), acc);
    }
    dH[node * kH + f] = acc;
}

// per block of 256 nodes: partial dW[k][o] = sum_i bf(X_ik) dZ_io (dZ = dH o [Hout > 0]),
// and (row K of the partial) db[o] = sum_i dZ_io.  Every sum runs over the block's nodes in
// order.  The nodes pass through LDS 64 at a time (their X rows rounded to bfloat16 and
// their dZ rows, each loaded once by coalesced reads); thread (q, o) = (tid / 64, tid % 64)
// then holds the sums of k = q*NK .. q*NK + NK - 1, reading the X entries as wavefront-wide
// broadcasts.
constexpr int kGradChunk = 64;   // nodes staged in LDS at a time

template <int K>
__global__ __launch_bounds__(256) void k_wgrad_part(int32_t n, const float *__restrict__ X, const float *__restrict__ dH,
                                                    const float *__restrict__ Hout, float *__restrict__ part)
{
    static_assert(K % 4 == 0, "four thread groups of K / 4 rows each");
    constexpr int NK = K / 4;
    __shared__ float sX[kGradChunk * K];
    __shared__ float sZ[kGradChunk * kH];
    const int t = threadIdx.x;
    const int o = t & 63;
    const int q = t >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * kNodeBlock;
    const int64_t i1 = (i0 + kNodeBlock) < n ? i0 + kNodeBlock : n;
    float *out = part + (int64_t)blockIdx.x * (K + 1) * kH;
    float acc[NK];
#pragma unroll
    for (int m = 0; m < NK; ++m) acc[m] = 0.f;
    float db = 0.f;
    for (int64_t c0 = i0; c0 < i1; c0 += kGradChunk) {
        const int cn = (int)((i1 - c0) < kGradChunk ? (i1 - c0) : kGradChunk);
        if (cn == kGradChunk) {
#pragma unroll
            for (int v = 0; v < (kGradChunk * K + 255) / 256; ++v) {
                const int u = t + 256 * v;
                if (u < kGradChunk * K) sX[u] = bfr(X[c0 * K + u]);
            }
#pragma unroll
            for (int v = 0; v < kGradChunk * kH / 256; ++v) {
                const int u = t + 256 * v;
                const int64_t gi = c0 * kH + u;
                const float h = Hout[gi], d = dH[gi];
                sZ[u] = h > 0.f ? d : 0.f;
            }
        } else {
            for (int u = t; u < cn * K; u += 256) sX[u] = bfr(X[c0 * K + u]);
            for (int u = t; u < cn * kH; u += 256) {
                const int64_t gi = c0 * kH + u;
                sZ[u] = Hout[gi] > 0.f ? dH[gi] : 0.f;
            }
        }
        __syncthreads();
        for (int r = 0; r < cn; ++r) {
            const float dz = sZ[r * kH + o];
            db += dz;
            const float *xr = sX + r * K + q * NK;
#pragma unroll
            for (int m = 0; m < NK; ++m) acc[m] = fmaf(xr[m], dz, acc[m]);
        }
        __syncthreads();
    }
    if (q == 0) out[K * kH + o] = db;
#pragma unroll
    for (int m = 0; m < NK; ++m) out[(q * NK + m) * kH + o] = acc[m];
}

// sum of nb partials in block order, the loads issued eight at a time
__device__ __forceinline__ float sum_parts(const float *__restrict__ part, int nb, int64_t stride, int64_t g)
{
    float acc = 0.f;
    int b = 0;
    for (; b + 8 <= nb; b += 8) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = part[(int64_t)(b + j) * stride + g];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc += v[j];
    }
    for (; b < nb; ++b) acc += part[(int64_t)b * stride + g];
    return acc;
}

// grad[off_w + k*64 + o] += sum_blocks part[b][k][o] (block order); grad[off_b + o] likewise
template <int K>
__global__ __launch_bounds__(256) void k_wgrad_reduce(int nb, const float *__restrict__ part, float *__restrict__ grad,
                                                      int off_w, int off_b)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= (int64_t)(K + 1) * kH) return;
    const float acc = sum_parts(part, nb, (int64_t)(K + 1) * kH, g);
    if (g < (int64_t)K * kH) grad[off_w + g] += acc;
    else if (off_b >= 0) grad[off_b + (g - K * kH)] += acc;
}

// readout parameter gradients: per node block, dwu[f] = sum du_i bf(h_if), dbu = sum du_i;
// per edge block, dqv[f] = sum dv_k bf(h_if) bf(h_jf), dbv = sum dv_k.  Each sum in node
// (edge) order; the operands of eight nodes (edges) are loaded ahead of their arithmetic.
__global__ __launch_bounds__(64) void k_readout_grad_part(int32_t n, int64_t nnz, const int32_t *__restrict__ rows,
                                                          const int32_t *__restrict__ ci, const float *__restrict__ H,
                                                          const float *__restrict__ du, const float *__restrict__ dv,
                                                          int nblk, float *__restrict__ part)
{
    const int f = threadIdx.x;
    float *out = part + (int64_t)blockIdx.x * 2 * (kH + 1);
    if ((int)blockIdx.x < nblk) {
        const int64_t i0 = (int64_t)blockIdx.x * kNodeBlock;
        const int64_t i1 = (i0 + kNodeBlock) < n ? i0 + kNodeBlock : n;
        float a = 0.f, b = 0.f;
        int64_t i = i0;
        for (; i + 8 <= i1; i += 8) {
            float d[8], h[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                d[j] = du[i + j];
                h[j] = H[(i + j) * kH + f];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                a = fmaf(d[j], bfr(h[j]), a);
                b += d[j];
            }
        }
        for (; i < i1; ++i) {
            a = fmaf(du[i], bfr(H[i * kH + f]), a);
            b += du[i];
        }
        out[f] = a;
        if (f == 0) out[kH] = b;
        out[kH + 1 + f] = 0.f;
        if (f == 0) out[2 * kH + 1] = 0.f;
    } else {
        const int64_t e0 = (int64_t)(blockIdx.x - nblk) * kEdgeBlock;
        const int64_t e1 = (e0 + kEdgeBlock) < nnz ? e0 + kEdgeBlock : nnz;
        float a = 0.f, b = 0.f;
        int64_t e = e0;
        for (; e + 8 <= e1; e += 8) {
            int32_t ri[8], cj[8];
            float d[8], hi[8], hj[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                ri[j] = rows[e + j];
                cj[j] = ci[e + j];
                d[j] = dv[e + j];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                hi[j] = H[(int64_t)ri[j] * kH + f];
                hj[j] = H[(int64_t)cj[j] * kH + f];
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (ri[j] == cj[j]) continue;
                a = fmaf(d[j], bfr(hi[j]) * bfr(hj[j]), a);
                b += d[j];
            }
        }
        for (; e < e1; ++e) {
            const int64_t i = rows[e], j = ci[e];
            if (i == j) continue;
            a = fmaf(dv[e], bfr(H[i * kH + f]) * bfr(H[j * kH + f]), a);
            b += dv[e];
        }
        out[f] = 0.f;
        if (f == 0) out[kH] = 0.f;
        out[kH + 1 + f] = a;
        if (f == 0) out[2 * kH + 1] = b;
    }
}

__global__ __launch_bounds__(256) void k_readout_grad_reduce(int nparts, const float *__restrict__ part,
                                                             float *__restrict__ grad)
{
    const int g = threadIdx.x;
    if (g >= 2 * (kH + 1)) return;
    const float acc = sum_parts(part, nparts, 2 * (kH + 1), g);
    // layout of a part: [wu(64), bu, qv(64), bv]
    if (g < kH) grad[OFF_WU + g] += acc;
    else if (g == kH) grad[OFF_BU] += acc;
    else if (g < 2 * kH + 1) grad[OFF_QV + (g - kH - 1)] += acc;
    else grad[OFF_BV] += acc;
}

__global__ __launch_bounds__(256) void k_fill_f(int64_t n, float *__restrict__ p, float v)
{
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

__global__ __launch_bounds__(256) void k_adam(int n, float *__restrict__ theta, const float *__restrict__ grad,
                                              float *__restrict__ m, float *__restrict__ v, float lr, float b1,
                                              float b2, float eps, float gscale, float c1, float c2)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i] * gscale;
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    theta[i] = theta[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline unsigned nb256(int64_t n)
{
    const int64_t b = (n + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b < 65536 ? b : 65536));
}

void graph_free(mp_graph *g)
{
    if (!g) return;
    if (g->d_arena) (void)hipFree(g->d_arena);
    delete g;
}

// The graph's buffers, carved from one allocation (one hipMalloc / hipFree per graph
// instead of one per buffer): a first pass with base == nullptr sizes the arena, a
// second assigns each buffer its 256-byte aligned offset.
struct Carver {
    char *base;
    size_t off;
    template <typename T>
    void take(T **p, size_t count)
    {
        off = (off + 255) & ~(size_t)255;
        if (base) *p = reinterpret_cast<T *>(base + off);
        off += sizeof(T) * (count > 0 ? count : 1);
    }
};

void graph_layout(mp_graph *g, Carver &c)
{
    const size_t n = (size_t)g->n, nnz = (size_t)g->nnz;
    const size_t nh = n * kH;
    const size_t wpart = (size_t)(g->nblk > 0 ? g->nblk : 1) * (kH + 1) * kH;
    const size_t rpart = (size_t)(g->nblk + g->eblk) * 2 * (kH + 1);
    c.take(&g->d_rows, nnz);
    c.take(&g->d_rev, nnz);
    c.take(&g->d_w, nnz);
    c.take(&g->d_f, n * kF);
    c.take(&g->d_minv, n);
    for (int l = 0; l < 4; ++l) c.take(&g->d_H[l], nh);
    for (int l = 1; l < 4; ++l) c.take(&g->d_Mg[l], nh);
    c.take(&g->d_u, n);
    c.take(&g->d_v, nnz);
    c.take(&g->d_c, nnz);
    c.take(&g->d_du, n);
    c.take(&g->d_dv, nnz);
    c.take(&g->d_dH, nh);
    c.take(&g->d_dH2, nh);
    c.take(&g->d_dMg, nh);
    c.take(&g->d_wpart, wpart > rpart ? wpart : rpart);
    c.take(&g->d_vec, (size_t)5 * n);
    c.take(&g->d_dpart, (size_t)2 * ((n + 4095) / 4096) + 2);
    c.take(&g->d_M, nnz);
    c.take(&g->d_bad, 1);
}

// forward pass of graph g: activations, readouts, c and M (in g->d_M)
mp_status mpnn_forward(const mp_mpnn *net, mp_graph *g, hipStream_t s)
{
    const int32_t n = g->n;
    const float *th = net->d_theta;
    const unsigned nodes4 = (unsigned)((n + 3) / 4);
    hipLaunchKernelGGL((k_dense<kF, false>), dim3(nodes4), dim3(256), 0, s, n, g->d_f, th + OFF_W0, nullptr, nullptr,
                       th + OFF_B0, g->d_H[0]);
    for (int l = 1; l <= 3; ++l) {
        hipLaunchKernelGGL(k_aggregate, dim3((unsigned)(((int64_t)n * kH + 255) / 256)), dim3(256), 0, s, n, g->row_ptr,
                           g->col_idx, g->d_w, g->d_H[l - 1], nullptr, g->d_Mg[l]);
        hipLaunchKernelGGL(k_dense_mfma, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s, n, g->d_H[l - 1], th + off_ws(l),
                           g->d_Mg[l], th + off_wn(l), th + off_b(l), g->d_H[l]);
    }
    hipLaunchKernelGGL(k_readout, dim3(nb256(g->nnz > n ? g->nnz : n)), dim3(256), 0, s, n, g->nnz, g->d_rows,
                       g->col_idx, g->d_H[3], th, g->d_u, g->d_v);
    hipLaunchKernelGGL(k_assemble, dim3(nb256(n)), dim3(256), 0, s, n, g->row_ptr, g->col_idx, g->d_u, g->d_v,
                       g->d_w, g->d_minv, g->d_c, g->d_M);
    MP_HIP_TRY(hipGetLastError());
    return MP_OK;
}

}  // namespace mpk

extern "C" {

mp_status mp_mpnn_param_count(int32_t *count)
{
    mpk::clear_error();
    if (!count) return mpk::fail(MP_ERR_INVALID_ARG, "count is NULL");
    *count = mpk::N_PARAMS;
    return MP_OK;
}

mp_status mp_mpnn_create(int32_t hidden, mp_mpnn **out)
{
    using namespace mpk;
    clear_error();
    if (!out) return fail(MP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (hidden != kH) return fail(MP_ERR_UNSUPPORTED, "hidden width must be %d", kH);
    mp_mpnn *p = new (std::nothrow) mp_mpnn;
    if (!p) return fail(MP_ERR_NO_MEMORY, "allocation failed");
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&p->d_theta), sizeof(float) * 4 * N_PARAMS);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipMalloc(network)");
    }
    p->d_grad = p->d_theta + N_PARAMS;
    p->d_m = p->d_grad + N_PARAMS;
    p->d_v = p->d_m + N_PARAMS;
    e = hipMemset(p->d_theta, 0, sizeof(float) * 4 * N_PARAMS);
    if (e != hipSuccess) {
        (void)hipFree(p->d_theta);
        delete p;
        return hip_fail(e, "hipMemset(network)");
    }
    *out = p;
    return MP_OK;
}

mp_status mp_mpnn_destroy(mp_mpnn *net)
{
    mpk::clear_error();
    if (net) {
        if (net->d_theta) (void)hipFree(net->d_theta);
        delete net;
    }
    return MP_OK;
}

static mp_status mpnn_copy(mp_mpnn *net, int which, float *host, bool to_device, bool adam_reset)
{
    using namespace mpk;
    clear_error();
    if (!net || !host) return fail(MP_ERR_INVALID_ARG, "NULL argument");
    float *dst = which == 0 ? net->d_theta : net->d_grad;
    if (to_device) {
        MP_HIP_TRY(hipMemcpy(dst, host, sizeof(float) * N_PARAMS, hipMemcpyHostToDevice));
        if (adam_reset) MP_HIP_TRY(hipMemset(net->d_m, 0, sizeof(float) * 2 * N_PARAMS));
    } else {
        MP_HIP_TRY(hipMemcpy(host, dst, sizeof(float) * N_PARAMS, hipMemcpyDeviceToHost));
    }
    return MP_OK;
}

mp_status mp_mpnn_set_params(mp_mpnn *net, const float *host_params)
{
    return mpnn_copy(net, 0, const_cast<float *>(host_params), true, true);
}

mp_status mp_mpnn_get_params(const mp_mpnn *net, float *host_params)
{
    return mpnn_copy(const_cast<mp_mpnn *>(net), 0, host_params, false, false);
}

mp_status mp_mpnn_get_grads(const mp_mpnn *net, float *host_grads)
{
    return mpnn_copy(const_cast<mp_mpnn *>(net), 1, host_grads, false, false);
}

mp_status mp_mpnn_zero_grads(mp_mpnn *net, void *stream)
{
    mpk::clear_error();
    if (!net) return mpk::fail(MP_ERR_INVALID_ARG, "net is NULL");
    hipLaunchKernelGGL(mpk::k_fill_f, dim3(mpk::nb256(mpk::N_PARAMS)), dim3(256), 0, static_cast<hipStream_t>(stream),
                       (int64_t)mpk::N_PARAMS, net->d_grad, 0.f);
    MP_HIP_TRY(hipGetLastError());
    return MP_OK;
}

mp_status mp_graph_create(const mp_csr *A, const double *a, void *stream, mp_graph **out)
{
    using namespace mpk;
    clear_error();
    if (!out) return fail(MP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    mp_status st = check_csr(A);
    if (st != MP_OK) return st;
    if (A->n_rows != A->n_cols) return fail(MP_ERR_INVALID_ARG, "matrix must be square");
    if (A->nnz > 0 && !a) return fail(MP_ERR_INVALID_ARG, "a is NULL");
    mp_graph *g = new (std::nothrow) mp_graph;
    if (!g) return fail(MP_ERR_NO_MEMORY, "allocation failed");
    const int32_t n = A->n_rows;
    const int64_t nnz = A->nnz;
    g->n = n;
    g->nnz = nnz;
    g->row_ptr = A->row_ptr;
    g->col_idx = A->col_idx;
    g->a = a;
    g->nblk = (int32_t)((n + kNodeBlock - 1) / kNodeBlock);
    g->eblk = (int32_t)((nnz + kEdgeBlock - 1) / kEdgeBlock);
    Carver sizer{nullptr, 0};
    graph_layout(g, sizer);
    {
        const hipError_t e = hipMalloc(&g->d_arena, sizer.off);
        if (e != hipSuccess) {
            g->d_arena = nullptr;
            graph_free(g);
            return hip_fail(e, "hipMalloc");
        }
    }
    Carver carver{static_cast<char *>(g->d_arena), 0};
    graph_layout(g, carver);
    int32_t *d_bad = g->d_bad;
    int32_t h_bad = INT32_MAX;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (st == MP_OK) {
        hipError_t e = hipMemcpyAsync(d_bad, &h_bad, sizeof(int32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess && n > 0) {
            hipLaunchKernelGGL(k_g_diag, dim3(nb256(n)), dim3(256), 0, s, n, A->row_ptr, A->col_idx, a, g->d_minv,
                               g->d_rows, d_bad);
            hipLaunchKernelGGL(k_g_edges, dim3(nb256(n)), dim3(256), 0, s, n, A->row_ptr, A->col_idx, a, g->d_minv,
                               g->d_w, g->d_f, g->d_rev, d_bad);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipMemcpyAsync(&h_bad, d_bad, sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = hip_fail(e, "graph set-up");
        else if (h_bad != INT32_MAX)
            st = fail(MP_ERR_INVALID_ARG,
                      "row %d has no positive diagonal, a positive off-diagonal entry or an entry without its transpose",
                      h_bad);
    }
    if (st != MP_OK) {
        graph_free(g);
        return st;
    }
    *out = g;
    return MP_OK;
}

mp_status mp_graph_destroy(mp_graph *g)
{
    mpk::clear_error();
    mpk::graph_free(g);
    return MP_OK;
}

mp_status mp_mpnn_forward(const mp_mpnn *net, mp_graph *g, double *m_values, void *stream)
{
    using namespace mpk;
    clear_error();
    if (!net || !g) return fail(MP_ERR_INVALID_ARG, "NULL argument");
    if (g->nnz > 0 && !m_values) return fail(MP_ERR_INVALID_ARG, "m_values is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (g->n == 0) return MP_OK;
    mp_status st = mpnn_forward(net, g, s);
    if (st != MP_OK) return st;
    MP_HIP_TRY(hipMemcpyAsync(m_values, g->d_M, sizeof(double) * g->nnz, hipMemcpyDeviceToDevice, s));
    return MP_OK;
}

mp_status mp_mpnn_loss_grad(mp_mpnn *net, mp_graph *g, const double *r, const double *e, int32_t npairs,
                            double *loss_host, void *stream)
{
    using namespace mpk;
    clear_error();
    if (!net || !g || npairs < 1 || (g->n > 0 && (!r || !e)))
        return fail(MP_ERR_INVALID_ARG, "mp_mpnn_loss_grad: NULL argument or npairs < 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int32_t n = g->n;
    if (n == 0) return MP_OK;
    if (npairs > n) return fail(MP_ERR_INVALID_ARG, "mp_mpnn_loss_grad: npairs = %d exceeds n = %d", npairs, n);
    mp_status st = mpnn_forward(net, g, s);
    if (st != MP_OK) return st;
    hipLaunchKernelGGL(k_fill_f, dim3(nb256(n)), dim3(256), 0, s, (int64_t)n, g->d_du, 0.f);
    hipLaunchKernelGGL(k_fill_f, dim3(nb256(g->nnz)), dim3(256), 0, s, g->nnz, g->d_dv, 0.f);
    double *y = g->d_vec, *Ad = g->d_vec + n, *Ae = g->d_vec + 2 * (int64_t)n, *out = g->d_vec + 3 * (int64_t)n;
    const int m = (n + 4095) / 4096;
    double *pdd = g->d_dpart, *pee = g->d_dpart + m;
    std::vector<double> losses((size_t)npairs * 2);
    for (int p = 0; p < npairs; ++p) {
        const double *rp_ = r + (int64_t)p * n, *ep = e + (int64_t)p * n;
        // d = M r - e, Ad, Ae (binary64, rows sequential; A = hi of the DD values)
        hipLaunchKernelGGL(k_spmv64, dim3(nb256(n)), dim3(256), 0, s, n, g->row_ptr, g->col_idx, g->d_M, rp_, ep, y);
        hipLaunchKernelGGL(k_spmv64, dim3(nb256(n)), dim3(256), 0, s, n, g->row_ptr, g->col_idx, g->a, y, nullptr, Ad);
        hipLaunchKernelGGL(k_spmv64, dim3(nb256(n)), dim3(256), 0, s, n, g->row_ptr, g->col_idx, g->a, ep, nullptr, Ae);
        hipLaunchKernelGGL(k_dot64, dim3(m), dim3(256), 0, s, n, y, Ad, pdd);
        hipLaunchKernelGGL(k_dot64, dim3(m), dim3(256), 0, s, n, ep, Ae, pee);
        hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, pdd, pee, m, out + 2 * p);
        hipLaunchKernelGGL(k_assemble_bwd, dim3(nb256(n)), dim3(256), 0, s, n, g->row_ptr, g->col_idx, Ad, out + 2 * p,
                           rp_, g->d_minv, g->d_u, g->d_v, g->d_w, g->d_du, g->d_dv);
        MP_HIP_TRY(hipGetLastError());
    }
    // readouts -> dH3 and readout parameter gradients
    const float *th = net->d_theta;
    float *grad = net->d_grad;
    const unsigned nh = (unsigned)(((int64_t)n * kH + 255) / 256);
    hipLaunchKernelGGL(k_readout_bwd, dim3(nh), dim3(256), 0, s, n, g->row_ptr, g->col_idx, g->d_rev, g->d_H[3], th,
                       g->d_du, g->d_dv, g->d_dH);
    hipLaunchKernelGGL(k_readout_grad_part, dim3(g->nblk + g->eblk), dim3(64), 0, s, n, g->nnz, g->d_rows, g->col_idx,
                       g->d_H[3], g->d_du, g->d_dv, g->nblk, g->d_wpart);
    hipLaunchKernelGGL(k_readout_grad_reduce, dim3(1), dim3(256), 0, s, g->nblk + g->eblk, g->d_wpart, grad);
    const unsigned nodes4 = (unsigned)((n + 3) / 4);
    float *dH = g->d_dH, *dH2 = g->d_dH2;
    for (int l = 3; l >= 1; --l) {
        // weight gradients of layer l (Ws with X = H[l-1], Wn with X = Mg[l]); bias with the first
        hipLaunchKernelGGL((k_wgrad_part<kH>), dim3(g->nblk), dim3(256), 0, s, n, g->d_H[l - 1], dH, g->d_H[l],
                           g->d_wpart);
        hipLaunchKernelGGL((k_wgrad_reduce<kH>), dim3((unsigned)(((kH + 1) * kH + 255) / 256)), dim3(256), 0, s,
                           g->nblk, g->d_wpart, grad, off_ws(l), off_b(l));
        hipLaunchKernelGGL((k_wgrad_part<kH>), dim3(g->nblk), dim3(256), 0, s, n, g->d_Mg[l], dH, g->d_H[l],
                           g->d_wpart);
        hipLaunchKernelGGL((k_wgrad_reduce<kH>), dim3((unsigned)(((kH + 1) * kH + 255) / 256)), dim3(256), 0, s,
                           g->nblk, g->d_wpart, grad, off_wn(l), -1);
        // input gradients: dH[l-1] = dZ Ws^T + aggregate(dZ Wn^T)
        hipLaunchKernelGGL(k_dense_bwd_x_mfma, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s, n, dH, g->d_H[l],
                           th + off_ws(l), dH2,
                           th + off_wn(l), g->d_dMg);
        hipLaunchKernelGGL(k_aggregate, dim3(nh), dim3(256), 0, s, n, g->row_ptr, g->col_idx, g->d_w, g->d_dMg, dH2, dH);
    }
    hipLaunchKernelGGL((k_wgrad_part<kF>), dim3(g->nblk), dim3(256), 0, s, n, g->d_f, dH, g->d_H[0], g->d_wpart);
    hipLaunchKernelGGL((k_wgrad_reduce<kF>), dim3((unsigned)(((kF + 1) * kH + 255) / 256)), dim3(256), 0, s, g->nblk,
                       g->d_wpart, grad, OFF_W0, OFF_B0);
    MP_HIP_TRY(hipGetLastError());
    if (loss_host) {
        MP_HIP_TRY(hipMemcpyAsync(losses.data(), out, sizeof(double) * 2 * npairs, hipMemcpyDeviceToHost, s));
        MP_HIP_TRY(hipStreamSynchronize(s));
        for (int p = 0; p < npairs; ++p) loss_host[p] = losses[2 * p];
    }
    return MP_OK;
}

mp_status mp_mpnn_adam_step(mp_mpnn *net, float lr, float beta1, float beta2, float eps, float grad_scale,
                            int32_t step, void *stream)
{
    using namespace mpk;
    clear_error();
    if (!net || step < 1) return fail(MP_ERR_INVALID_ARG, "bad argument");
    const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3((N_PARAMS + 255) / 256), dim3(256), 0, static_cast<hipStream_t>(stream), N_PARAMS,
                       net->d_theta, net->d_grad, net->d_m, net->d_v, lr, beta1, beta2, eps, grad_scale, c1, c2);
    MP_HIP_TRY(hipGetLastError());
    return MP_OK;
}

}  // extern "C"
