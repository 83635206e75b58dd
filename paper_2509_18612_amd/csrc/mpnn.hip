// Learned starting magnitudes: a 3-layer message-passing network over node degree
// features, with hand-written forward and backward kernels (bfloat16 weights, float32
// accumulation) and an Adam update. Not part of the paper's method (which is training-free);
// it proposes per-node magnitudes y_v in (0, 1) that multiply the importance-based signs
// of Sec. 4.1 to form a starting mean (DECO_INIT_LEARNED).
//
//   f_v = [d_v / dbar, m_v / dbar, log(1 + d_v) - log(1 + dbar)]   (per graph dbar)
//   h <- relu(h Ws_k + a Wn_k + b_k),  a_v = mean_{u in N(v)} h_u,  k = 1..3 (3->64->64->64)
//   y = sigmoid(h wo + bo),  L = mean_v (y_v - t_v)^2
//
// Parameters are one packed float32 vector (deco.h gives the layout); the forward pass
// rounds them to bfloat16 when staging them in LDS. Weight gradients are reduced in two
// deterministic stages (per-workgroup partial sums, then a fixed-order sum).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "../../include/deco.h"

namespace {

constexpr int kH = 64, kIn = 3;
// packed parameter offsets
constexpr int oWs1 = 0, oWn1 = oWs1 + kIn * kH, oB1 = oWn1 + kIn * kH;
constexpr int oWs2 = oB1 + kH, oWn2 = oWs2 + kH * kH, oB2 = oWn2 + kH * kH;
constexpr int oWs3 = oB2 + kH, oWn3 = oWs3 + kH * kH, oB3 = oWn3 + kH * kH;
constexpr int oWo = oB3 + kH, oBo = oWo + kH, kNumParams = oBo + 1;
constexpr int kRedBlocks = 128;  // workgroups of the first reduction stage

__device__ __forceinline__ float rbf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

__device__ __forceinline__ int graph_of(const int* goff, int G, long long v) {
  int lo = 0, hi = G;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (goff[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

// features (n x 4, last column 0)
__global__ void k_features(long long n, const int* rp, const int* ci, const int* goff, int G, float* F) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int g = graph_of(goff, G, v);
  const long long r0 = goff[g], r1 = goff[g + 1];
  double dbar = (double)(rp[r1] - rp[r0]) / (double)(r1 - r0);
  if (dbar <= 0.0) dbar = 1.0;
  const int d = rp[v + 1] - rp[v];
  double s = 0.0;
  for (int k = rp[v]; k < rp[v + 1]; ++k) s += (double)(rp[ci[k] + 1] - rp[ci[k]]);
  const double m = d > 0 ? s / d : 0.0;
  F[v * 4 + 0] = (float)(d / dbar);
  F[v * 4 + 1] = (float)(m / dbar);
  F[v * 4 + 2] = (float)(log1p((double)d) - log1p(dbar));
  F[v * 4 + 3] = 0.0f;
}

// A[v, :] = mean_{u in N(v)} H[u, :] (or the adjoint-sum form with per-source scaling)
// H, A: n x ld, first `dim` columns used. scale_src: multiply H[u] by 1/d_u (adjoint).
__global__ void k_aggregate(long long n, const int* rp, const int* ci, const float* H, int ld, int dim, float* A,
                            int adjoint) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * dim) return;
  const long long v = i / dim;
  const int j = (int)(i % dim);
  const int beg = rp[v], end = rp[v + 1];
  float s = 0.0f;
  for (int k = beg; k < end; ++k) {
    const int u = ci[k];
    const float hu = H[(long long)u * ld + j];
    s += adjoint ? hu / (float)(rp[u + 1] - rp[u]) : hu;
  }
  A[v * ld + j] = adjoint ? s : (end > beg ? s / (float)(end - beg) : 0.0f);
}

// y = sigmoid(H3 wo + bo); with a target, also dz = dL/dz and the per-row loss terms.
__global__ void k_head(long long n, const float* H3, const float* P, const float* t, float* y, float* dz,
                       double* lossterm, double inv_n) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  float z = rbf16(P[oBo]);
  for (int j = 0; j < kH; ++j) z = fmaf(H3[v * kH + j], rbf16(P[oWo + j]), z);
  const double yy = 1.0 / (1.0 + exp(-(double)z));
  y[v] = (float)yy;
  if (t) {
    const double e = yy - (double)t[v];
    lossterm[v] = e * e;
    dz[v] = (float)(2.0 * e * inv_n * yy * (1.0 - yy));
  }
}

// dH3 = dz wo^T (times relu mask of Pre3) -> dPre3
__global__ void k_head_back(long long n, const float* dz, const float* P, const float* Pre3, float* dPre) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * kH) return;
  const long long v = i / kH;
  const int j = (int)(i % kH);
  dPre[i] = Pre3[i] > 0.0f ? dz[v] * rbf16(P[oWo + j]) : 0.0f;
}

// Stage 1 of the head's weight gradient G[i][j] = sum_v X[v][i] D[v][j] (i < dim, plus i ==
// dim for a column of ones, i.e. the bias), per workgroup over a contiguous row range.
__global__ __launch_bounds__(256) void k_wgrad_partial(long long n, const float* Xm, int ldx, int dim,
                                                       const float* D, int ldd, int dout, float* part) {
  const long long per = (n + gridDim.x - 1) / gridDim.x;
  const long long r0 = blockIdx.x * per, r1 = r0 + per < n ? r0 + per : n;
  const int total = (dim + 1) * dout;
  for (int o = threadIdx.x; o < total; o += blockDim.x) {
    const int i = o / dout, j = o % dout;
    float s = 0.0f;
    for (long long v = r0; v < r1; ++v) s = fmaf(i < dim ? Xm[v * ldx + i] : 1.0f, D[v * ldd + j], s);
    part[(size_t)blockIdx.x * total + o] = s;
  }
}

// Stage 2: fixed-order sum of the partials into gW (dim x dout) and gb (dout).
__global__ void k_wgrad_final(const float* part, int nparts, int dim, int dout, float* gW, float* gb) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = (dim + 1) * dout;
  if (o >= total) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += part[(size_t)p * total + o];
  const int i = o / dout, j = o % dout;
  if (i < dim)
    gW[i * dout + j] = (float)s;
  else if (gb)
    gb[j] = (float)s;
}

// ---------------------------------------------------------------- matrix-core versions
// The three dense products of a layer run on the matrix cores with float32 operands and
// accumulation (v_mfma_f32_32x32x2f32): the weights are the bfloat16-rounded parameters, the
// activations stay float32. Operand layout of one 32 x 32 x 2 step for lane (lo, hi) =
// (lane % 32, lane / 32): A[lo][k0 + hi] and B[k0 + hi][lo]; element r of the 16 results is
// row 8 (r / 4) + 4 hi + r % 4, column lo.
typedef float f32x16_t __attribute__((ext_vector_type(16)));
constexpr int kTile = 64;      // nodes per tile
constexpr int kWgBlocks = 256; // workgroups (partial sums) of a weight gradient

__device__ __forceinline__ int mfma_row(int r, int hi) { return 8 * (r >> 2) + 4 * hi + (r & 3); }

// Pre = [H | A] [Ws; Wn] + b, Hout = relu(Pre): each workgroup stages the concatenated
// weights once and walks tiles of 64 nodes; wave (wm, wn) computes nodes 32 wm.. and
// outputs 32 wn.. of a tile.
__global__ __launch_bounds__(256) void k_linear_mfma(long long n, const float* H, const float* A, int ld, int dim,
                                                     const float* P, int ows, int own, int ob, float* Pre,
                                                     float* Hout) {
  __shared__ float sw[2 * kH][kH];
  __shared__ float sb[kH];
  __shared__ float sx[kTile][2 * kH + 1];  // odd row stride: a column read hits 32 banks
  const int K = 2 * dim, Kp = (K + 1) & ~1;
  for (int i = threadIdx.x; i < Kp * kH; i += blockDim.x) {
    const int k = i / kH, j = i % kH;
    float w = 0.0f;
    if (k < dim)
      w = rbf16(P[ows + k * kH + j]);
    else if (k < K)
      w = rbf16(P[own + (k - dim) * kH + j]);
    sw[k][j] = w;
  }
  for (int i = threadIdx.x; i < kH; i += blockDim.x) sb[i] = rbf16(P[ob + i]);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, lo = lane & 31, hi = lane >> 5;
  const int wm = wv >> 1, wn = wv & 1;
  const long long ntiles = (n + kTile - 1) / kTile;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long v0 = tile * kTile;
    __syncthreads();  // the previous tile is consumed (first pass: the weights are staged)
    for (int i = threadIdx.x; i < kTile * Kp; i += blockDim.x) {
      const int r = i / Kp, k = i % Kp;
      const long long v = v0 + r;
      float x = 0.0f;
      if (v < n) {
        if (k < dim)
          x = H[v * ld + k];
        else if (k < K)
          x = A[v * ld + (k - dim)];
      }
      sx[r][k] = x;
    }
    __syncthreads();
    f32x16_t acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    for (int k0 = 0; k0 < Kp; k0 += 2)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(sx[wm * 32 + lo][k0 + hi], sw[k0 + hi][wn * 32 + lo], acc, 0, 0,
                                                 0);
    const int j = wn * 32 + lo;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const long long v = v0 + wm * 32 + mfma_row(r, hi);
      if (v < n) {
        const float y = acc[r] + sb[j];
        Pre[v * kH + j] = y;
        Hout[v * kH + j] = fmaxf(y, 0.0f);
      }
    }
  }
}

// T1 = dPre Ws^T, T2 = dPre Wn^T for a hidden layer (64 inputs): B = [Ws^T | Wn^T] (64 x 128);
// wave (wm, wn) computes nodes 32 wm.. of T1 (wn = 0) or T2 (wn = 1) as two 32-column blocks.
__global__ __launch_bounds__(256) void k_dinput_mfma(long long n, const float* dPre, const float* P, int ows, int own,
                                                     float* T1, float* T2) {
  __shared__ float sw[kH][2 * kH];
  __shared__ float sx[kTile][kH + 1];
  for (int e = threadIdx.x; e < kH * 2 * kH; e += blockDim.x) {
    const int j = e / (2 * kH), c = e % (2 * kH);
    sw[j][c] = c < kH ? rbf16(P[ows + c * kH + j]) : rbf16(P[own + (c - kH) * kH + j]);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, lo = lane & 31, hi = lane >> 5;
  const int wm = wv >> 1, wn = wv & 1;
  float* T = wn ? T2 : T1;
  const long long ntiles = (n + kTile - 1) / kTile;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long v0 = tile * kTile;
    __syncthreads();
    for (int i = threadIdx.x; i < kTile * kH; i += blockDim.x) {
      const int r = i / kH, k = i % kH;
      const long long v = v0 + r;
      sx[r][k] = v < n ? dPre[v * kH + k] : 0.0f;
    }
    __syncthreads();
    f32x16_t acc[2];
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;
    for (int k0 = 0; k0 < kH; k0 += 2) {
      const float a = sx[wm * 32 + lo][k0 + hi];
#pragma unroll
      for (int q = 0; q < 2; ++q)
        acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, sw[k0 + hi][wn * kH + q * 32 + lo], acc[q], 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const long long v = v0 + wm * 32 + mfma_row(r, hi);
        if (v < n) T[v * kH + q * 32 + lo] = acc[q][r];
      }
  }
}

// Stage 1 of the weight gradients of a layer: per workgroup, over its chunks of 64 nodes,
// Gs = Hin^T D and Gn = Ain^T D (M = 2 dim rows, 64 columns, as 32 x 32 blocks spread over the
// waves) and gb = column sums of D (fixed order). part[block] holds (2 dim + 1) x 64 floats:
// rows k < dim Gs, dim <= k < 2 dim Gn, row 2 dim gb.
__global__ __launch_bounds__(256) void k_wgrad_mfma(long long n, const float* Hin, const float* Ain, int ld, int dim,
                                                    const float* D, float* part) {
  __shared__ float sx[kTile][2 * kH + 1];
  __shared__ float sd[kTile][kH];
  const int M = 2 * dim, mb = (M + 31) / 32, Mp = 32 * mb, nblk = 2 * mb;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, lo = lane & 31, hi = lane >> 5;
  f32x16_t acc[2];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[q][r] = 0.0f;
  float bsum = 0.0f;
  const long long nchunks = (n + kTile - 1) / kTile;
  for (long long c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const long long v0 = c * kTile;
    __syncthreads();
    for (int i = threadIdx.x; i < kTile * Mp; i += blockDim.x) {
      const int r = i / Mp, k = i % Mp;
      const long long v = v0 + r;
      float x = 0.0f;
      if (v < n) {
        if (k < dim)
          x = Hin[v * ld + k];
        else if (k < M)
          x = Ain[v * ld + (k - dim)];
      }
      sx[r][k] = x;
    }
    for (int i = threadIdx.x; i < kTile * kH; i += blockDim.x) {
      const int r = i / kH, j = i % kH;
      const long long v = v0 + r;
      sd[r][j] = v < n ? D[v * kH + j] : 0.0f;
    }
    __syncthreads();
    if (threadIdx.x < kH)
      for (int r = 0; r < kTile; ++r) bsum += sd[r][threadIdx.x];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = wv + 4 * q;
      if (idx < nblk) {
        const int bm = idx >> 1, bn = idx & 1;
        for (int k0 = 0; k0 < kTile; k0 += 2)
          acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(sx[k0 + hi][bm * 32 + lo], sd[k0 + hi][bn * 32 + lo], acc[q],
                                                        0, 0, 0);
      }
    }
  }
  float* out = part + (size_t)blockIdx.x * (M + 1) * kH;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int idx = wv + 4 * q;
    if (idx < nblk) {
      const int bm = idx >> 1, bn = idx & 1;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = bm * 32 + mfma_row(r, hi);
        if (m < M) out[m * kH + bn * 32 + lo] = acc[q][r];
      }
    }
  }
  if (threadIdx.x < kH) out[M * kH + threadIdx.x] = bsum;
}

// Stage 2: fixed-order (double) sum of the partials into gWs, gWn (dim x 64) and gb (64).
__global__ void k_wgrad_final_layer(const float* part, int nparts, int dim, float* gWs, float* gWn, float* gb) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  const int total = (2 * dim + 1) * kH;
  if (o >= total) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += part[(size_t)p * total + o];
  const int m = o / kH, j = o % kH;
  if (m < dim)
    gWs[m * kH + j] = (float)s;
  else if (m < 2 * dim)
    gWn[(m - dim) * kH + j] = (float)s;
  else
    gb[j] = (float)s;
}

// dPre_prev = (T1 + aggT) * relu'(Pre_prev), where aggT was computed into Agg.
__global__ void k_combine(long long n, const float* T1, const float* Agg, const float* PrePrev, float* dPrev) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * kH) return;
  dPrev[i] = PrePrev[i] > 0.0f ? T1[i] + Agg[i] : 0.0f;
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, long long count, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  m[i] = b1 * m[i] + (1.0f - b1) * gi;
  v[i] = b2 * v[i] + (1.0f - b2) * gi * gi;
  p[i] -= lr * (m[i] / c1) / (sqrtf(v[i] / c2) + eps);
}

// t_v = sum_u w 1{z_u != z_v} / d_w(v)
__global__ void k_labels(long long n, const int* rp, const int* ci, const float* w, const uint8_t* z, float* t) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  double c = 0.0, d = 0.0;
  for (int k = rp[v]; k < rp[v + 1]; ++k) {
    const double wk = w ? w[k] : 1.0;
    d += wk;
    if (z[ci[k]] != z[v]) c += wk;
  }
  t[v] = d != 0.0 ? (float)(c / d) : 0.0f;
}

__global__ void k_sum_double(const double* x, long long n, double* out) {
  __shared__ double s[256];
  double a = 0.0;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) a += x[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

inline unsigned nb(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

struct Buffers {
  float *F, *A1, *P1, *H1, *A2, *P2, *H2, *A3, *P3, *H3, *y, *dz, *D3, *D2, *D1, *T1, *T2, *AG, *part, *goff;
  double *lt, *loss;
  size_t total;
};

Buffers carve(char* base, long long n) {
  Buffers b{};
  size_t off = 0;
  auto f = [&](size_t count) {
    float* p = base ? reinterpret_cast<float*>(base + off) : nullptr;
    off += (count * sizeof(float) + 255) / 256 * 256;
    return p;
  };
  b.F = f(n * 4);
  b.A1 = f(n * 4);
  float** hk[] = {&b.P1, &b.H1, &b.A2, &b.P2, &b.H2, &b.A3, &b.P3, &b.H3, &b.D3, &b.D2, &b.D1, &b.T1, &b.T2, &b.AG};
  for (auto p : hk) *p = f(n * kH);
  b.y = f(n);
  b.dz = f(n);
  b.part = f((size_t)kWgBlocks * (2 * kH + 1) * kH);  // also holds the head's kRedBlocks x (kH + 1)
  b.goff = f(2);
  b.lt = reinterpret_cast<double*>(f(2 * n));
  b.loss = reinterpret_cast<double*>(f(2));
  b.total = off;
  return b;
}

deco_status check(const deco_graph* g) {
  if (!g || g->n < 1 || !g->row_ptr || (g->nnz > 0 && !g->col_idx) || g->num_graphs < 1 ||
      (g->num_graphs > 1 && !g->graph_row_offset))
    return DECO_E_INVAL;
  return DECO_OK;
}

// Workgroups of the tiled dense kernels: one per 64-node tile, at most 1024 (each walks the
// rest, reusing its staged weights).
unsigned lin_grid(long long n) {
  const long long t = (n + kTile - 1) / kTile;
  return (unsigned)(t < 1024 ? t : 1024);
}

hipError_t forward(const deco_graph* g, const float* P, const Buffers& b, const int* goff, hipStream_t s) {
  const long long n = g->n;
  const int G = g->num_graphs;
  hipLaunchKernelGGL(k_features, dim3(nb(n, 256)), dim3(256), 0, s, n, g->row_ptr, g->col_idx, goff, G, b.F);
  // layer 1 (input dim 3, stored with row stride 4)
  hipLaunchKernelGGL(k_aggregate, dim3(nb(n * 4, 256)), dim3(256), 0, s, n, g->row_ptr, g->col_idx, b.F, 4, 4, b.A1, 0);
  const unsigned lg = lin_grid(n);
  hipLaunchKernelGGL(k_linear_mfma, dim3(lg), dim3(256), 0, s, n, b.F, b.A1, 4, kIn, P, oWs1, oWn1, oB1, b.P1, b.H1);
  hipLaunchKernelGGL(k_aggregate, dim3(nb(n * kH, 256)), dim3(256), 0, s, n, g->row_ptr, g->col_idx, b.H1, kH, kH, b.A2, 0);
  hipLaunchKernelGGL(k_linear_mfma, dim3(lg), dim3(256), 0, s, n, b.H1, b.A2, kH, kH, P, oWs2, oWn2, oB2, b.P2, b.H2);
  hipLaunchKernelGGL(k_aggregate, dim3(nb(n * kH, 256)), dim3(256), 0, s, n, g->row_ptr, g->col_idx, b.H2, kH, kH, b.A3, 0);
  hipLaunchKernelGGL(k_linear_mfma, dim3(lg), dim3(256), 0, s, n, b.H2, b.A3, kH, kH, P, oWs3, oWn3, oB3, b.P3, b.H3);
  return hipGetLastError();
}

// Forward-only layout (the allocation-free variant): one pre-activation buffer shared by
// the three layers (the forward pass only writes it), layer 3's input and output reuse
// layer 1's buffers once layer 2 has consumed them; 1,056 bytes per node plus 256.
Buffers carve_forward(char* base, long long n) {
  Buffers b{};
  size_t off = 0;
  auto f = [&](size_t count) {
    float* p = base ? reinterpret_cast<float*>(base + off) : nullptr;
    off += (count * sizeof(float) + 255) / 256 * 256;
    return p;
  };
  b.F = f(n * 4);
  b.A1 = f(n * 4);
  b.P1 = b.P2 = b.P3 = f(n * kH);
  b.H1 = b.H3 = f(n * kH);
  b.A2 = b.A3 = f(n * kH);
  b.H2 = f(n * kH);
  b.goff = f(2);
  b.total = off;
  return b;
}

__global__ void k_goff_single(int* goff, int n) {
  if (threadIdx.x == 0) {
    goff[0] = 0;
    goff[1] = n;
  }
}

// Scratch of deco_mpnn_forward_static: a file-scope device array, one copy per GPU for the
// life of the process. Host code reaches it only through the per-device address returned
// by hipGetSymbolAddress (the array's name is not a device address on the host).
constexpr size_t kStaticScratch = (size_t)32 << 20;
__device__ __align__(256) char scratch[kStaticScratch];
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mu;

// Address of this device's copy of the scratch array (looked up once per device, with
// the device current).
hipError_t static_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

const int* goff_of(const deco_graph* g, const Buffers& b, hipStream_t s, hipError_t* e) {
  if (g->graph_row_offset) return g->graph_row_offset;
  const int h[2] = {0, (int)g->n};
  *e = hipMemcpyAsync(b.goff, h, sizeof(h), hipMemcpyHostToDevice, s);
  if (*e == hipSuccess) *e = hipStreamSynchronize(s);
  return reinterpret_cast<const int*>(b.goff);
}

}  // namespace

extern "C" {

int32_t deco_mpnn_num_params(void) { return kNumParams; }

deco_status deco_mpnn_workspace_size(const deco_graph* g, size_t* bytes) {
  deco_status st = check(g);
  if (st) return st;
  if (!bytes) return DECO_E_INVAL;
  *bytes = carve(nullptr, g->n).total;
  return DECO_OK;
}

deco_status deco_mpnn_forward(const deco_graph* g, const float* params, float* y, void* workspace, size_t bytes,
                              void* stream) {
  deco_status st = check(g);
  if (st) return st;
  if (!params || !y || !workspace || bytes < carve(nullptr, g->n).total) return params && y ? DECO_E_NOMEM : DECO_E_INVAL;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const Buffers b = carve(reinterpret_cast<char*>(workspace), g->n);
  hipError_t e = hipSuccess;
  const int* goff = goff_of(g, b, s, &e);
  if (e == hipSuccess) e = forward(g, params, b, goff, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_head, dim3(nb(g->n, 256)), dim3(256), 0, s, (long long)g->n, b.H3, params, nullptr, y,
                       nullptr, nullptr, 0.0);
    e = hipGetLastError();
  }
  return e == hipSuccess ? DECO_OK : DECO_E_DEVICE;
}

deco_status deco_mpnn_forward_static(const deco_graph* g, const float* params, float* y, void* stream) {
  deco_status st = check(g);
  if (st) return st;
  if (!params || !y) return DECO_E_INVAL;
  if (carve_forward(nullptr, g->n).total > kStaticScratch) return DECO_E_UNSUPPORTED;
  void* base = nullptr;
  if (static_scratch(&base) != hipSuccess) return DECO_E_DEVICE;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const Buffers b = carve_forward(reinterpret_cast<char*>(base), g->n);
  const int* goff = g->graph_row_offset;
  if (!goff) {
    hipLaunchKernelGGL(k_goff_single, dim3(1), dim3(64), 0, s, reinterpret_cast<int*>(b.goff), (int)g->n);
    goff = reinterpret_cast<const int*>(b.goff);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = forward(g, params, b, goff, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_head, dim3(nb(g->n, 256)), dim3(256), 0, s, (long long)g->n, b.H3, params, nullptr, y,
                       nullptr, nullptr, 0.0);
    e = hipGetLastError();
  }
  return e == hipSuccess ? DECO_OK : DECO_E_DEVICE;
}

deco_status deco_mpnn_loss_grad(const deco_graph* g, const float* params, const float* target, float* grads,
                                double* loss, void* workspace, size_t bytes, void* stream) {
  deco_status st = check(g);
  if (st) return st;
  if (!params || !target || !grads || !workspace) return DECO_E_INVAL;
  if (bytes < carve(nullptr, g->n).total) return DECO_E_NOMEM;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const long long n = g->n;
  const Buffers b = carve(reinterpret_cast<char*>(workspace), n);
  hipError_t e = hipSuccess;
  const int* goff = goff_of(g, b, s, &e);
  if (e == hipSuccess) e = forward(g, params, b, goff, s);
  if (e != hipSuccess) return DECO_E_DEVICE;
  const int* rp = g->row_ptr;
  const int* ci = g->col_idx;
  hipLaunchKernelGGL(k_head, dim3(nb(n, 256)), dim3(256), 0, s, n, b.H3, params, target, b.y, b.dz, b.lt,
                     1.0 / (double)n);
  hipLaunchKernelGGL(k_sum_double, dim3(1), dim3(256), 0, s, b.lt, n, b.loss);
  // head: gwo = H3^T dz, gbo = sum dz
  hipLaunchKernelGGL(k_wgrad_partial, dim3(kRedBlocks), dim3(256), 0, s, n, b.H3, kH, kH, b.dz, 1, 1, b.part);
  hipLaunchKernelGGL(k_wgrad_final, dim3(nb(kH + 1, 256)), dim3(256), 0, s, b.part, kRedBlocks, kH, 1,
                     grads + oWo, grads + oBo);
  hipLaunchKernelGGL(k_head_back, dim3(nb(n * kH, 256)), dim3(256), 0, s, n, b.dz, params, b.P3, b.D3);
  // layer 3: inputs H2 (Ws3), A3 (Wn3)
  struct L { const float *Hin, *Ain, *PrePrev; int ldin, dim, ows, own, ob; float *D, *Dprev; };
  const L layers[3] = {{b.H2, b.A3, b.P2, kH, kH, oWs3, oWn3, oB3, b.D3, b.D2},
                       {b.H1, b.A2, b.P1, kH, kH, oWs2, oWn2, oB2, b.D2, b.D1},
                       {b.F, b.A1, nullptr, 4, kIn, oWs1, oWn1, oB1, b.D1, nullptr}};
  const long long nchunks = (n + kTile - 1) / kTile;
  const int wg = (int)(nchunks < kWgBlocks ? nchunks : kWgBlocks);
  for (const L& l : layers) {
    hipLaunchKernelGGL(k_wgrad_mfma, dim3(wg), dim3(256), 0, s, n, l.Hin, l.Ain, l.ldin, l.dim, l.D, b.part);
    hipLaunchKernelGGL(k_wgrad_final_layer, dim3(nb((2 * l.dim + 1) * kH, 256)), dim3(256), 0, s, b.part, wg, l.dim,
                       grads + l.ows, grads + l.own, grads + l.ob);
    if (l.Dprev) {
      hipLaunchKernelGGL(k_dinput_mfma, dim3(lin_grid(n)), dim3(256), 0, s, n, l.D, params, l.ows, l.own, b.T1,
                         b.T2);
      hipLaunchKernelGGL(k_aggregate, dim3(nb(n * kH, 256)), dim3(256), 0, s, n, rp, ci, b.T2, kH, kH, b.AG, 1);
      hipLaunchKernelGGL(k_combine, dim3(nb(n * kH, 256)), dim3(256), 0, s, n, b.T1, b.AG, l.PrePrev, l.Dprev);
    }
  }
  e = hipGetLastError();
  if (e == hipSuccess && loss) e = hipMemcpyAsync(loss, b.loss, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && loss) *loss /= (double)n;
  return e == hipSuccess ? DECO_OK : DECO_E_DEVICE;
}

deco_status deco_mpnn_adam(float* params, const float* grads, float* m, float* v, int32_t step, float lr,
                           void* stream) {
  if (!params || !grads || !m || !v || step < 1 || !(lr > 0.0f)) return DECO_E_INVAL;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(nb(kNumParams, 256)), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), params,
                     grads, m, v, (long long)kNumParams, lr, b1, b2, 1e-8f, c1, c2);
  return hipGetLastError() == hipSuccess ? DECO_OK : DECO_E_DEVICE;
}

deco_status deco_mpnn_labels(const deco_graph* g, const uint8_t* z, float* target, void* stream) {
  deco_status st = check(g);
  if (st) return st;
  if (!z || !target) return DECO_E_INVAL;
  hipLaunchKernelGGL(k_labels, dim3(nb(g->n, 256)), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                     (long long)g->n, g->row_ptr, g->col_idx, g->w, z, target);
  return hipGetLastError() == hipSuccess ? DECO_OK : DECO_E_DEVICE;
}

}  // extern "C"
