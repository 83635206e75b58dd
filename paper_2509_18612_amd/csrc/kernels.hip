// Device kernels of the DECO library for gfx950 (CDNA4, wave64).
//
// The hot kernel, k_step, performs one step of batched projected gradient ascent
// (Sec. 3.1 eq. (6)-(7), Sec. 3.2 lifted update) fused with the exact scoring of the
// iterate it reads (eq. (5) / lifted rounding, eq. (1)) and the running best of Alg. 1-2:
//
//   for every row v and initialisation b (all l components):
//     acc   = sum_{u in N(v)} w_vu X_t[u, i, b]           (float32, CSR order per sub-group)
//     X_t+1 = clip(X_t[v] + eta_b (cW acc + cD d_w(v) X_t[v]), -1, 1)
//     score += w_vu 1{z_t(v) != z_t(u)}                   (double, exact for integer w)
//
// Mapping: node-major X (row v holds all l*B values contiguously). A row is handled by a
// sub-group of Wc lanes, each lane owning VEC consecutive initialisations of a tile of
// Bt = Wc*VEC, for every component (16-byte loads). 'split' sub-groups share one row and
// split its neighbour list (long rows); a wave therefore covers 64/(Wc*split) rows. Work
// items (row range x initialisation tile) are grouped per XCD and walked by a persistent
// grid, so an XCD's L2 serves the gathers of its own rows / tile. Neighbour gathers are
// issued four at a time to keep loads in flight. The score partials stay in registers
// until the workgroup changes (graph, tile), then go through a wave reduction, an LDS
// reduction and one double atomic per initialisation into one of R replicated
// accumulators. The last workgroup of the launch (ticket counter) turns the sums into
// cuts, updates the running best and the improvement mask, and advances the step counter.
// The cut bits of an improved step are folded into best_bits by the next launch, row by
// row, before that launch overwrites the same bit slot.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace deco {

namespace {

__device__ __forceinline__ float bf2f(uint32_t h16) { return __uint_as_float(h16 << 16); }

// float32 -> bfloat16, round to nearest even (inputs are finite, |x| <= 1 here).
__device__ __forceinline__ uint32_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

template <typename T, int VEC>
struct VecIO;

template <>
struct VecIO<float, 4> {
  static __device__ __forceinline__ void load(const float* p, float (&o)[4]) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
  static __device__ __forceinline__ void store(float* p, const float (&o)[4]) {
    *reinterpret_cast<float4*>(p) = make_float4(o[0], o[1], o[2], o[3]);
  }
};

template <>
struct VecIO<float, 1> {
  static __device__ __forceinline__ void load(const float* p, float (&o)[1]) { o[0] = *p; }
  static __device__ __forceinline__ void store(float* p, const float (&o)[1]) { *p = o[0]; }
};

template <>
struct VecIO<uint16_t, 8> {
  static __device__ __forceinline__ void load(const uint16_t* p, float (&o)[8]) {
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    o[0] = bf2f(v.x & 0xFFFFu);
    o[1] = bf2f(v.x >> 16);
    o[2] = bf2f(v.y & 0xFFFFu);
    o[3] = bf2f(v.y >> 16);
    o[4] = bf2f(v.z & 0xFFFFu);
    o[5] = bf2f(v.z >> 16);
    o[6] = bf2f(v.w & 0xFFFFu);
    o[7] = bf2f(v.w >> 16);
  }
  static __device__ __forceinline__ void store(uint16_t* p, const float (&o)[8]) {
    uint4 v;
    v.x = f2bf(o[0]) | (f2bf(o[1]) << 16);
    v.y = f2bf(o[2]) | (f2bf(o[3]) << 16);
    v.z = f2bf(o[4]) | (f2bf(o[5]) << 16);
    v.w = f2bf(o[6]) | (f2bf(o[7]) << 16);
    *reinterpret_cast<uint4*>(p) = v;
  }
};

template <>
struct VecIO<uint16_t, 1> {
  static __device__ __forceinline__ void load(const uint16_t* p, float (&o)[1]) { o[0] = bf2f(*p); }
  static __device__ __forceinline__ void store(uint16_t* p, const float (&o)[1]) {
    *p = (uint16_t)f2bf(o[0]);
  }
};

// Rounding of one initialisation from its l component values (float32, order i = 0..l-1).
template <int L>
__device__ __forceinline__ bool side_of(const float (&x)[L], int lifted) {
  if (!lifted) return x[0] > 0.0f;
  float s = 0.0f;
#pragma unroll
  for (int i = 0; i < L; ++i) s = s + x[i];
  return s >= 0.0f;
}

constexpr int kWaves = 4;  // waves per workgroup
constexpr int kUnroll = 4; // neighbour gathers in flight per sub-group

template <typename T, int VEC, int L, bool UNIT>
__global__ __launch_bounds__(256) void k_step(StepArgs a) {
  __shared__ double s_red[kWaves][64 * VEC];
  __shared__ int s_last;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int Wc = a.Wc;
  const int split = a.split;
  const int gw = Wc * split;
  const int lc = lane & (Wc - 1);
  const int sg = (lane / Wc) & (split - 1);
  const int rs = lane / gw;
  const int rpw = 64 / gw;

  const long long t = a.ctrl->t;
  const bool do_score = a.force_score || (t % a.ctrl->score_every) == 0;
  const int pend = a.ctrl->pending_slot;
  const int par = (int)(t & 1);
  const T* __restrict__ X = reinterpret_cast<const T*>(a.x[par]);
  T* __restrict__ Y = reinterpret_cast<T*>(a.x[par ^ 1]);
  uint8_t* __restrict__ bw = a.bits[par];
  const uint8_t* bm = pend >= 0 ? a.bits[pend] : nullptr;
  const int C = a.C, B = a.B, NBY = a.NBY;
  const int Bt = Wc * VEC;
  const int gb = VEC >= 8 ? 1 : (8 / VEC < Wc ? 8 / VEC : Wc);  // lanes per cut-bit byte

  const int xcd = blockIdx.x & 7;
  const int kb = blockIdx.x >> 3;
  const int nbx = ((int)gridDim.x - xcd + 7) >> 3;
  const int it0 = a.seg[xcd], it1 = a.seg[xcd + 1];

  double sc[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) sc[e] = 0.0;
  float eta_l[VEC];
  int cg = -1, cbt = -1;

  for (int it = it0 + kb;; it += nbx) {
    const bool have = it < it1;
    int4 item = make_int4(0, 0, -1, -1);
    if (have) item = a.items[it];
    if (do_score && cg >= 0 && (!have || item.z != cg || item.w != cbt)) {
      // flush the partial scores of (cg, cbt): wave, then workgroup, then one atomic
#pragma unroll
      for (int e = 0; e < VEC; ++e)
        for (int s = Wc; s < 64; s <<= 1) sc[e] += __shfl_xor(sc[e], s);
      if (lane < Wc) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) s_red[wv][lane * VEC + e] = sc[e];
      }
      __syncthreads();
      for (int j = tid; j < Bt; j += 256) {
        double v = s_red[0][j];
#pragma unroll
        for (int q = 1; q < kWaves; ++q) v += s_red[q][j];
        if (v != 0.0) {
          double* dst = a.acc + ((size_t)(blockIdx.x % a.R) * a.G + cg) * B + cbt * Bt + j;
          unsafeAtomicAdd(dst, v);
        }
      }
      __syncthreads();
#pragma unroll
      for (int e = 0; e < VEC; ++e) sc[e] = 0.0;
    }
    if (!have) break;
    cg = item.z;
    cbt = item.w;
    const int bl = cbt * Bt + lc * VEC;  // first initialisation of this lane
#pragma unroll
    for (int e = 0; e < VEC; ++e) eta_l[e] = a.eta[bl + e];

    for (int rb = item.x + wv * rpw; rb < item.y; rb += kWaves * rpw) {
      const int row = rb + rs;
      const bool valid = row < item.y;
      int beg = 0, end = 0;
      float xv[L][VEC];
      if (valid) {
        beg = a.rp[row];
        end = a.rp[row + 1];
#pragma unroll
        for (int i = 0; i < L; ++i)
          VecIO<T, VEC>::load(X + (size_t)row * C + (size_t)i * B + bl, xv[i]);
      } else {
#pragma unroll
        for (int i = 0; i < L; ++i)
#pragma unroll
          for (int e = 0; e < VEC; ++e) xv[i][e] = 0.0f;
      }
      bool zv[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        float g[L];
#pragma unroll
        for (int i = 0; i < L; ++i) g[i] = xv[i][e];
        zv[e] = side_of<L>(g, a.lifted);
      }
      float acc[L][VEC];
#pragma unroll
      for (int i = 0; i < L; ++i)
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[i][e] = 0.0f;

      for (int k = beg + sg; k < end; k += split * kUnroll) {
        int u[kUnroll];
        float wk[kUnroll];
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) {
          const int kk = k + q * split;
          const bool ok = kk < end;
          u[q] = ok ? a.ci[kk] : -1;
          wk[q] = ok ? (UNIT ? 1.0f : a.w[kk]) : 0.0f;
        }
        float xu[kUnroll][L][VEC];
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) {
          if (u[q] >= 0) {
#pragma unroll
            for (int i = 0; i < L; ++i)
              VecIO<T, VEC>::load(X + (size_t)u[q] * C + (size_t)i * B + bl, xu[q][i]);
          } else {
#pragma unroll
            for (int i = 0; i < L; ++i)
#pragma unroll
              for (int e = 0; e < VEC; ++e) xu[q][i][e] = 0.0f;
          }
        }
#pragma unroll
        for (int q = 0; q < kUnroll; ++q) {
#pragma unroll
          for (int i = 0; i < L; ++i)
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
              if (UNIT)
                acc[i][e] += xu[q][i][e];
              else
                acc[i][e] = fmaf(wk[q], xu[q][i][e], acc[i][e]);
            }
        }
        if (do_score) {
#pragma unroll
          for (int q = 0; q < kUnroll; ++q) {
            if (u[q] >= 0) {
#pragma unroll
              for (int e = 0; e < VEC; ++e) {
                float g[L];
#pragma unroll
                for (int i = 0; i < L; ++i) g[i] = xu[q][i][e];
                if (side_of<L>(g, a.lifted) != zv[e]) sc[e] += (double)wk[q];
              }
            }
          }
        }
      }
      // combine the sub-groups that split this row's neighbours
      for (int s = Wc; s < gw; s <<= 1) {
#pragma unroll
        for (int i = 0; i < L; ++i)
#pragma unroll
          for (int e = 0; e < VEC; ++e) acc[i][e] += __shfl_xor(acc[i][e], s);
      }
      const bool lead = valid && sg == 0;
      if (a.do_update && lead) {
        const float dwv = (a.cD != 0.0f) ? a.dw[row] : 0.0f;
#pragma unroll
        for (int i = 0; i < L; ++i) {
          float y[VEC];
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            float g = a.cW * acc[i][e];
            if (a.cD != 0.0f) g = fmaf(a.cD * dwv, xv[i][e], g);
            float v = fmaf(eta_l[e], g, xv[i][e]);
            y[e] = fminf(1.0f, fmaxf(-1.0f, v));
          }
          VecIO<T, VEC>::store(Y + (size_t)row * C + (size_t)i * B + bl, y);
        }
      }
      // cut bits of X_t: assemble bytes across the gb lanes that share one
      uint32_t byte = 0;
#pragma unroll
      for (int e = 0; e < VEC; ++e) byte |= (zv[e] ? 1u : 0u) << e;
      byte <<= (lc * VEC) & 7;
      for (int s = 1; s < gb; s <<= 1) byte |= __shfl_xor(byte, s);
      if (lead && (lc % gb) == 0) {
        const size_t bi = (size_t)row * NBY + (bl >> 3);
        if (pend >= 0) {
          const uint32_t m = a.mask[cg * NBY + (bl >> 3)];
          if (m) {
            const uint32_t old = bm[bi];
            const uint32_t bb = a.best_bits[bi];
            a.best_bits[bi] = (uint8_t)((bb & ~m) | (old & m));
          }
        }
        if (do_score) bw[bi] = (uint8_t)byte;
      }
    }
  }

  // ---- last workgroup: cuts, running best, improvement mask, step counter
  __threadfence();
  __syncthreads();
  if (tid == 0) {
    const unsigned prev = atomicAdd(&a.ctrl->ticket, 1u);
    s_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  const int GB = a.G * B;
  if (do_score) {
    const int chunk = B < 8 ? B : 8;
    for (int base = 0; base < GB; base += 256) {
      const int idx = base + tid;
      const bool in = idx < GB;
      bool imp = false;
      if (in) {
        double s = 0.0;
        for (int r = 0; r < a.R; ++r) {
          double* p = a.acc + (size_t)r * GB + idx;
          s += __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_store(p, 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const double cut = 0.5 * s;
        a.cur_cut[idx] = cut;
        if (a.trace) a.trace[(size_t)(t % a.trace_cap) * GB + idx] = cut;
        imp = cut > a.best_cut[idx];
        if (imp) {
          a.best_cut[idx] = cut;
          a.best_step[idx] = (int)t;
        }
      }
      const unsigned long long bal = __ballot(imp);
      if (in && (idx % chunk) == 0) {
        const int g = idx / B, b = idx % B;
        a.mask[g * NBY + (b >> 3)] = (uint8_t)((bal >> lane) & ((1ull << chunk) - 1ull));
      }
    }
  }
  if (tid == 0) {
    a.ctrl->pending_slot = do_score ? par : -1;
    if (a.do_update) a.ctrl->t = t + 1;
    a.ctrl->ticket = 0u;
  }
}

template <typename T, int VEC>
hipError_t step_dispatch_l(const StepArgs& a, bool unit, int grid, hipStream_t s) {
  dim3 g(grid), b(256);
#define DECO_LAUNCH(LL)                                                           \
  if (unit)                                                                       \
    hipLaunchKernelGGL((k_step<T, VEC, LL, true>), g, b, 0, s, a);                \
  else                                                                            \
    hipLaunchKernelGGL((k_step<T, VEC, LL, false>), g, b, 0, s, a);
  switch (a.L) {
    case 1: DECO_LAUNCH(1); break;
    case 2: DECO_LAUNCH(2); break;
    case 3: DECO_LAUNCH(3); break;
    case 4: DECO_LAUNCH(4); break;
    default: return hipErrorInvalidValue;
  }
#undef DECO_LAUNCH
  return hipGetLastError();
}

// ------------------------------------------------------------------ graph validation
// flags: bit0 bad column / self-loop / unsorted, bit1 asymmetric, bit2 non-finite weight,
// bit3 edge leaving its graph, bit4 non-integral weight (information only).
__global__ void k_validate(long long n, const int* rp, const int* ci, const float* w,
                           const int* goff, int G, float* dw, int* flags) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int lo = 0, hi = G;  // graph of row v: goff[g] <= v < goff[g+1]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (goff[mid] <= v) lo = mid; else hi = mid;
  }
  const long long g0 = goff[lo], g1 = goff[lo + 1];
  const int beg = rp[v], end = rp[v + 1];
  int f = 0;
  float s = 0.0f;
  int prev = -1;
  for (int k = beg; k < end; ++k) {
    const int u = ci[k];
    const float wk = w ? w[k] : 1.0f;
    if (u < 0 || u >= n || u == v || u <= prev) {
      f |= 1;
      break;
    }
    prev = u;
    if (u < g0 || u >= g1) f |= 8;
    if (!isfinite(wk)) f |= 4;
    if (wk != floorf(wk) || fabsf(wk) > 1048576.0f) f |= 16;
    s += wk;
    // mirror entry: binary search v in row u
    int a0 = rp[u], a1 = rp[u + 1] - 1;
    bool found = false;
    while (a0 <= a1) {
      const int m = (a0 + a1) >> 1;
      const int cm = ci[m];
      if (cm == v) {
        found = (w == nullptr) || (w[m] == wk);
        break;
      }
      if (cm < v) a0 = m + 1; else a1 = m - 1;
    }
    if (!found) f |= 2;
  }
  if (dw) dw[v] = s;
  if (f) atomicOr(flags, f);
}

// ------------------------------------------------------------------ state reset
__global__ void k_reset(StepArgs a, double* acc_all, long long acc_count, int score_every) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long GB = (long long)a.G * a.B;
  if (i < acc_count) acc_all[i] = 0.0;
  if (i < GB) {
    a.best_cut[i] = -__builtin_inf();
    a.best_step[i] = -1;
    a.cur_cut[i] = -__builtin_inf();
  }
  if (i < (long long)a.G * a.NBY) a.mask[i] = 0;
  if (i == 0) {
    a.ctrl->ticket = 0u;
    a.ctrl->pending_slot = -1;
    a.ctrl->t = 0;
    a.ctrl->score_every = score_every;
    a.ctrl->pad = 0;
  }
}

// Fold the pending improvement mask into best_bits (idempotent until the slot is reused).
__global__ void k_merge(StepArgs a, long long n, const int* goff) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int pend = a.ctrl->pending_slot;
  if (pend < 0 || i >= n * a.NBY) return;
  const long long row = i / a.NBY;
  const int by = (int)(i % a.NBY);
  int lo = 0, hi = a.G;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (goff[mid] <= row) lo = mid; else hi = mid;
  }
  const uint32_t m = a.mask[lo * a.NBY + by];
  if (m) {
    const uint32_t old = a.bits[pend][i];
    const uint32_t bb = a.best_bits[i];
    a.best_bits[i] = (uint8_t)((bb & ~m) | (old & m));
  }
}

__global__ void k_fill(float* p, int n, float v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ starting points
__device__ __forceinline__ void draw4(unsigned long long seed, uint32_t a0, uint32_t a1,
                                      uint32_t purpose, uint32_t batch, uint32_t (&r)[4]) {
  r[0] = a0;
  r[1] = a1;
  r[2] = purpose;
  r[3] = batch;
  philox4x32_10(r, (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ __forceinline__ double u24(uint32_t r) { return (double)(r >> 8) * (1.0 / 16777216.0); }

__device__ __forceinline__ void store_x(void* X, long long idx, int dtype, double y) {
  if (y > 1.0) y = 1.0;
  if (y < -1.0) y = -1.0;
  const float f = (float)y;
  if (dtype == 0)
    reinterpret_cast<float*>(X)[idx] = f;
  else
    reinterpret_cast<uint16_t*>(X)[idx] = (uint16_t)f2bf(f);
}

__device__ __forceinline__ int graph_of(const int* goff, int G, long long v) {
  int lo = 0, hi = G;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (goff[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

// IDI phase 1: important nodes draw p = +-1, others 0 (Sec. 4.1).
__global__ void k_idi_sign(InitArgs a) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n * a.C) return;
  const long long v = i / a.C;
  const int c = (int)(i % a.C);
  const int g = graph_of(a.goff, a.G, v);
  const double d = (double)(a.rp[v + 1] - a.rp[v]);
  int8_t p = 0;
  if (d > a.thr[g]) {
    uint32_t r[4];
    draw4(a.seed, (uint32_t)v, (uint32_t)c, kIdiSign, a.batch, r);
    p = (r[0] >> 31) ? 1 : -1;
  }
  a.scratch[i] = p;
}

// All mean-based starts: X = Proj((h + sd * eps) / scale) with h by kind.
__global__ void k_init(InitArgs a) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n * a.C) return;
  const long long v = i / a.C;
  const int c = (int)(i % a.C);
  if (a.l_active) {
    const int comp = c / a.B, b = c % a.B;
    if (comp >= a.l_active[b]) {
      store_x(a.X, i, a.dtype, 0.0);
      return;
    }
  }
  uint32_t r[4];
  if (a.kind == 1) {  // uniform
    draw4(a.seed, (uint32_t)v, (uint32_t)c, kUniform, a.batch, r);
    store_x(a.X, i, a.dtype, 2.0 * u24(r[0]) - 1.0);
    return;
  }
  double h = 0.0;
  if (a.kind == 2) {  // DUI
    const int g = graph_of(a.goff, a.G, v);
    const int dl = a.delta[g];
    const double half = dl > 0 ? 1.0 - (double)(a.rp[v + 1] - a.rp[v]) / (double)dl : 1.0;
    draw4(a.seed, (uint32_t)v, (uint32_t)c, kDui, a.batch, r);
    h = (2.0 * u24(r[0]) - 1.0) * half;
  } else if (a.kind == 3) {  // IDI
    const int8_t p = a.scratch[i];
    if (p != 0) {
      h = (double)p;
    } else {
      double aa = 0.0, bb = 0.0;
      for (int k = a.rp[v]; k < a.rp[v + 1]; ++k) {
        const int8_t pu = a.scratch[(long long)a.ci[k] * a.C + c];
        const double wk = a.w ? (double)a.w[k] : 1.0;
        if (pu > 0) aa += wk;
        if (pu < 0) bb += wk;
      }
      if (aa == bb) {
        draw4(a.seed, (uint32_t)v, (uint32_t)c, kIdiTie, a.batch, r);
        h = (r[0] >> 31) ? 1.0 : -1.0;
      } else {
        h = aa < bb ? 1.0 : -1.0;
      }
    }
  } else if (a.kind == 4) {  // mean from a cut vector
    h = a.mean_z[v] ? 1.0 : -1.0;
  }
  double eps = 0.0;
  if (a.sd != 0.0) {
    draw4(a.seed, (uint32_t)v, (uint32_t)c, kGauss, a.batch, r);
    const double u1 = ((double)(r[0] >> 8) + 1.0) * (1.0 / 16777216.0);
    const double u2 = u24(r[1]);
    eps = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
  store_x(a.X, i, a.dtype, (h + a.sd * eps) / a.scale);
}

__global__ void k_convert_user(const void* x0, void* X, long long count, int dtype,
                               const int* l_active, int C, int B, int* nonfinite) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float f;
  if (dtype == 0) {
    f = reinterpret_cast<const float*>(x0)[i];
  } else {
    f = bf2f(reinterpret_cast<const uint16_t*>(x0)[i]);
  }
  if (!isfinite(f)) {
    atomicOr(nonfinite, 1);
    f = 0.0f;
  }
  f = fminf(1.0f, fmaxf(-1.0f, f));
  if (l_active) {
    const int c = (int)(i % C);
    if (c / B >= l_active[c % B]) f = 0.0f;
  }
  if (dtype == 0)
    reinterpret_cast<float*>(X)[i] = f;
  else
    reinterpret_cast<uint16_t*>(X)[i] = (uint16_t)f2bf(f);
}

__global__ void k_philox_test(uint32_t c1, uint32_t c2, uint32_t c3, unsigned long long seed,
                              int count, uint32_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint32_t r[4] = {(uint32_t)i, c1, c2, c3};
  philox4x32_10(r, (uint32_t)seed, (uint32_t)(seed >> 32));
  for (int j = 0; j < 4; ++j) out[(size_t)i * 4 + j] = r[j];
}

inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

int native_vec(int dtype) { return dtype == 0 ? 4 : 8; }

hipError_t launch_step(const StepArgs& a, int dtype, int vec, bool unit, int grid,
                       hipStream_t s) {
  if (dtype == 0) {
    if (vec == 4) return step_dispatch_l<float, 4>(a, unit, grid, s);
    if (vec == 1) return step_dispatch_l<float, 1>(a, unit, grid, s);
  } else {
    if (vec == 8) return step_dispatch_l<uint16_t, 8>(a, unit, grid, s);
    if (vec == 1) return step_dispatch_l<uint16_t, 1>(a, unit, grid, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_validate(long long n, const int* rp, const int* ci, const float* w,
                           const int* goff, int G, float* dw, int* flags, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, ci, w, goff, G,
                     dw, flags);
  return hipGetLastError();
}

hipError_t launch_reset(StepArgs a, double* acc_all, long long acc_count, int score_every,
                        hipStream_t s) {
  long long m = acc_count;
  const long long GB = (long long)a.G * a.B;
  if (GB > m) m = GB;
  if ((long long)a.G * a.NBY > m) m = (long long)a.G * a.NBY;
  if (m < 1) m = 1;
  hipLaunchKernelGGL(k_reset, dim3(blocks_for(m, 256)), dim3(256), 0, s, a, acc_all, acc_count,
                     score_every);
  return hipGetLastError();
}

hipError_t launch_merge(StepArgs a, long long n, const int* goff, hipStream_t s) {
  const long long m = n * a.NBY;
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_merge, dim3(blocks_for(m, 256)), dim3(256), 0, s, a, n, goff);
  return hipGetLastError();
}

hipError_t launch_fill_eta(float* eta, int B, float v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(B, 256)), dim3(256), 0, s, eta, B, v);
  return hipGetLastError();
}

hipError_t launch_init(const InitArgs& a, hipStream_t s) {
  const long long m = a.n * a.C;
  if (m <= 0) return hipSuccess;
  if (a.kind == 3) {
    hipLaunchKernelGGL(k_idi_sign, dim3(blocks_for(m, 256)), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_init, dim3(blocks_for(m, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_convert_user(const void* x0, void* X, long long count, int dtype,
                               const int* l_active, int C, int B, int* nonfinite,
                               hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert_user, dim3(blocks_for(count, 256)), dim3(256), 0, s, x0, X, count,
                     dtype, l_active, C, B, nonfinite);
  return hipGetLastError();
}

hipError_t launch_philox_test(uint32_t c1, uint32_t c2, uint32_t c3, unsigned long long seed,
                              int count, uint32_t* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox_test, dim3(blocks_for(count, 256)), dim3(256), 0, s, c1, c2, c3,
                     seed, count, out);
  return hipGetLastError();
}

}  // namespace deco
