// Resident step kernel: T steps of projected gradient ascent (Sec. 3.1 eq. (6)-(7)) with the
// rounding (eq. (5), or the lifted rule for l = 1), the exact cut (eq. (1)) and the running
// best of Alg. 1 for every scored iterate, in one launch, with each workgroup's share of X held
// in LDS for all T steps.
//
// Columns (initialisations) never interact in a step: column b of X_{t+1} depends only on
// column b of X_t. So a workgroup that owns one graph's rows and a tile of BT columns can run
// every step of those columns by itself: X_t and X_{t+1} of its tile sit in LDS (two
// buffers), the neighbour gathers read LDS, the graph structure comes from L2 (every
// workgroup of a graph reads the same CSR), and the cut of each of its columns is a
// workgroup reduction. No workgroup waits for another, so the launch needs no grid barrier
// and any number of workgroups may be in flight. The kernel applies when 2 n_g BT elements of
// the storage type fit the LDS budget (small and medium graphs, unlifted or l = 1).
//
// Work item i: {graph, first row, end row, first column}. Thread j of the workgroup owns a
// contiguous block of rows holding about 1/256 of the graph's slots (rows plus edges), so its
// column indices stream from one contiguous stretch of the CSR; it sums each row's neighbours
// in CSR order (the oracle's order) in batches of 8 loads, updates the row into the other
// buffer, and counts w 1{z_v != z_u} per column. The running best
// (cut, step and the sides of the best iterate) stays in LDS and registers during the launch
// and is written back at the end; the trace and the current cut are written per scored step.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "internal.h"

namespace deco {
namespace {

constexpr int kRThreads = 256;

__device__ __forceinline__ float r_bf2f(uint32_t h16) { return __uint_as_float(h16 << 16); }

typedef float r_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 r_bf16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t r_pack_bf16(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((r_f32x2{lo, hi}), r_bf16x2));
}

// BT consecutive elements of the storage type <-> float32.
template <typename T, int BT>
struct RowIO {
  static __device__ __forceinline__ void load(const T* p, float (&o)[BT]) {
    if constexpr (sizeof(T) == 4) {
      if constexpr (BT % 4 == 0) {
#pragma unroll
        for (int q = 0; q < BT / 4; ++q) {
          const float4 v = reinterpret_cast<const float4*>(p)[q];
          o[4 * q] = v.x;
          o[4 * q + 1] = v.y;
          o[4 * q + 2] = v.z;
          o[4 * q + 3] = v.w;
        }
      } else if constexpr (BT == 2) {
        const float2 v = *reinterpret_cast<const float2*>(p);
        o[0] = v.x;
        o[1] = v.y;
      } else {
        o[0] = *reinterpret_cast<const float*>(p);
      }
    } else {
      if constexpr (BT % 8 == 0) {
#pragma unroll
        for (int q = 0; q < BT / 8; ++q) {
          const uint4 v = reinterpret_cast<const uint4*>(p)[q];
          const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            o[8 * q + 2 * k] = r_bf2f(w[k] & 0xFFFFu);
            o[8 * q + 2 * k + 1] = r_bf2f(w[k] >> 16);
          }
        }
      } else if constexpr (BT == 4) {
        const uint2 v = *reinterpret_cast<const uint2*>(p);
        o[0] = r_bf2f(v.x & 0xFFFFu);
        o[1] = r_bf2f(v.x >> 16);
        o[2] = r_bf2f(v.y & 0xFFFFu);
        o[3] = r_bf2f(v.y >> 16);
      } else if constexpr (BT == 2) {
        const uint32_t v = *reinterpret_cast<const uint32_t*>(p);
        o[0] = r_bf2f(v & 0xFFFFu);
        o[1] = r_bf2f(v >> 16);
      } else {
        o[0] = r_bf2f(*reinterpret_cast<const uint16_t*>(p));
      }
    }
  }
  // float32 -> storage (bfloat16: round to nearest even, as the step kernel)
  static __device__ __forceinline__ void store(T* p, const float (&o)[BT]) {
    if constexpr (sizeof(T) == 4) {
#pragma unroll
      for (int c = 0; c < BT; ++c) reinterpret_cast<float*>(p)[c] = o[c];
    } else {
      if constexpr (BT == 1) {
        *reinterpret_cast<uint16_t*>(p) = (uint16_t)(r_pack_bf16(o[0], 0.0f) & 0xFFFFu);
      } else {
#pragma unroll
        for (int c = 0; c < BT; c += 2) reinterpret_cast<uint32_t*>(p)[c / 2] = r_pack_bf16(o[c], o[c + 1]);
      }
    }
  }
};

// Column partials of a workgroup: butterfly inside each wave, then the waves in order.
template <typename S, int BT>
__device__ __forceinline__ void block_sums(S (&v)[BT], S* s_red, int tid) {
#pragma unroll
  for (int c = 0; c < BT; ++c)
    for (int o = 32; o > 0; o >>= 1) v[c] += __shfl_xor(v[c], o);
  if ((tid & 63) == 0) {
#pragma unroll
    for (int c = 0; c < BT; ++c) s_red[(tid >> 6) * BT + c] = v[c];
  }
}

// WM: 0 unit weights (int counts), 1 integer weights (int counts), 2 real weights (double).
template <typename T, int BT, int WM>
__global__ __launch_bounds__(kRThreads) void k_resident(StepArgs a, const int4* __restrict__ items, int max_rows,
                                                        int steps) {
  using S = typename std::conditional<WM == 2, double, int>::type;
  extern __shared__ __align__(16) unsigned char r_smem[];
  __shared__ S s_red[(kRThreads / 64) * BT];
  __shared__ double s_best[BT];
  __shared__ int s_bstep[BT];
  __shared__ int s_imp[BT];
  __shared__ int s_any, s_ever;
  const int tid = threadIdx.x;
  const int4 it = items[blockIdx.x];
  const int g = it.x, r0 = it.y, r1 = it.z, c0 = it.w;
  const int nr = r1 - r0;
  T* buf0 = reinterpret_cast<T*>(r_smem);
  T* buf1 = buf0 + (size_t)max_rows * BT;
  uint32_t* s_bb = reinterpret_cast<uint32_t*>(buf1 + (size_t)max_rows * BT);
  const int nbw = (nr * BT + 31) >> 5;  // words of best bits
  const long long t0 = a.ctrl->t;
  const int every = a.ctrl->score_every;
  const size_t B = (size_t)a.B;

  // X_t0 of the tile into buffer 0; running best of the tile's columns
  const T* X0 = reinterpret_cast<const T*>(a.x[t0 & 1]);
  for (int i = tid; i < nr; i += kRThreads) {
    float v[BT];
    RowIO<T, BT>::load(X0 + (size_t)(r0 + i) * B + c0, v);
    RowIO<T, BT>::store(buf0 + (size_t)i * BT, v);
  }
  for (int i = tid; i < nbw; i += kRThreads) s_bb[i] = 0u;
  if (tid < BT) {
    s_best[tid] = a.best_cut[(size_t)g * B + c0 + tid];
    s_bstep[tid] = a.best_step[(size_t)g * B + c0 + tid];
    s_imp[tid] = 0;
  }
  if (tid == 0) s_ever = 0;
  float eta[BT], ecw[BT];
#pragma unroll
  for (int c = 0; c < BT; ++c) {
    eta[c] = a.eta[c0 + c];
    ecw[c] = eta[c] * a.cW;
  }
  const bool lifted = a.lifted != 0;
  int ever = 0;  // columns improved during this launch (bit c)
  // this thread's rows [rb, re): slot offsets S(v) = (rp[v] - rp[r0]) + (v - r0) split evenly
  int rb, re;
  {
    const long long E = (long long)(a.rp[r1] - a.rp[r0]) + nr;
    auto first_row = [&](int j) {
      const long long target = E * j / kRThreads;
      int lo = r0, hi = r1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((long long)(a.rp[mid] - a.rp[r0]) + (mid - r0) < target) lo = mid + 1; else hi = mid;
      }
      return lo;
    };
    rb = first_row(tid);
    re = tid + 1 < kRThreads ? first_row(tid + 1) : r1;
  }
  __syncthreads();

  for (int s = 0; s < steps; ++s) {
    const long long t = t0 + s;
    const bool do_score = (t % every) == 0;
    const T* cur = (s & 1) ? buf1 : buf0;
    T* nxt = (s & 1) ? buf0 : buf1;
    S cnt[BT];
#pragma unroll
    for (int c = 0; c < BT; ++c) cnt[c] = 0;
    int k1 = a.rp[rb];
    for (int v = rb; v < re; ++v) {
      const int i = v - r0;
      float xv[BT], acc[BT];
      RowIO<T, BT>::load(cur + (size_t)i * BT, xv);
      uint32_t zv = 0;
#pragma unroll
      for (int c = 0; c < BT; ++c) {
        acc[c] = 0.0f;
        zv |= (uint32_t)(lifted ? xv[c] >= 0.0f : xv[c] > 0.0f) << c;
      }
      const int k0 = k1;
      k1 = a.rp[v + 1];
      // neighbours in CSR order, 8 index loads in flight at a time
      for (int kb = k0; kb < k1; kb += 8) {
        const int nb = k1 - kb < 8 ? k1 - kb : 8;
        int uu[8];
        float ww[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          uu[q] = q < nb ? a.ci[kb + q] - r0 : 0;
          ww[q] = (WM == 0 || q >= nb) ? 1.0f : a.w[kb + q];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (q < nb) {
            const float wk = ww[q];
            float xu[BT];
            RowIO<T, BT>::load(cur + (size_t)uu[q] * BT, xu);
#pragma unroll
            for (int c = 0; c < BT; ++c) {
              if (WM == 0)
                acc[c] += xu[c];
              else
                acc[c] = fmaf(wk, xu[c], acc[c]);
            }
            if (do_score) {
#pragma unroll
              for (int c = 0; c < BT; ++c) {
                const bool zu = lifted ? xu[c] >= 0.0f : xu[c] > 0.0f;
                if (zu != (bool)((zv >> c) & 1u)) {
                  if (WM == 2)
                    cnt[c] += (S)wk;
                  else if (WM == 1)
                    cnt[c] += (S)(int)wk;
                  else
                    cnt[c] += 1;
                }
              }
            }
          }
        }
      }
      float y[BT];
#pragma unroll
      for (int c = 0; c < BT; ++c) {
        float x1;
        if (a.cD != 0.0f)
          x1 = fmaf(eta[c], fmaf(a.cD * a.dw[v], xv[c], a.cW * acc[c]), xv[c]);
        else
          x1 = fmaf(ecw[c], acc[c], xv[c]);
        y[c] = __builtin_amdgcn_fmed3f(x1, -1.0f, 1.0f);
      }
      RowIO<T, BT>::store(nxt + (size_t)i * BT, y);
    }
    if (do_score) block_sums<S, BT>(cnt, s_red, tid);
    __syncthreads();  // X_t+1 complete; wave partials ready
    if (do_score) {
      if (tid < BT) {
        S tot = 0;
#pragma unroll
        for (int q = 0; q < kRThreads / 64; ++q) tot += s_red[q * BT + tid];
        const double cut = 0.5 * (double)tot;
        const size_t idx = (size_t)g * B + c0 + tid;
        a.cur_cut[idx] = cut;
        if (a.trace) a.trace[(size_t)(t % a.trace_cap) * a.G * B + idx] = cut;
        const bool imp = cut > s_best[tid];
        if (imp) {
          s_best[tid] = cut;
          s_bstep[tid] = (int)t;
        }
        s_imp[tid] = imp ? 1 : 0;
      }
      if (tid == 0) s_any = 0;
      __syncthreads();
      if (tid < BT && s_imp[tid]) atomicOr(&s_any, 1 << tid);
      __syncthreads();
      const int m = s_any;
      ever |= m;
      if (m) {
        // sides of X_t (buffer cur) of this thread's rows into the best bits, improved columns
        for (int i = rb - r0; i < re - r0; ++i) {
          float xv[BT];
          RowIO<T, BT>::load(cur + (size_t)i * BT, xv);
#pragma unroll
          for (int c = 0; c < BT; ++c) {
            if ((m >> c) & 1) {
              const int bit = i * BT + c;
              const bool z = lifted ? xv[c] >= 0.0f : xv[c] > 0.0f;
              if (z)
                atomicOr(&s_bb[bit >> 5], 1u << (bit & 31));
              else
                atomicAnd(&s_bb[bit >> 5], ~(1u << (bit & 31)));
            }
          }
        }
      }
    }
  }
  __syncthreads();

  // X_{t0 + steps} back to global memory; running best and its sides
  const T* fin = (steps & 1) ? buf1 : buf0;
  T* Xo = reinterpret_cast<T*>(a.x[(t0 + steps) & 1]);
  for (int i = tid; i < nr; i += kRThreads) {
    float v[BT];
    RowIO<T, BT>::load(fin + (size_t)i * BT, v);
    RowIO<T, BT>::store(Xo + (size_t)(r0 + i) * B + c0, v);
  }
  if (tid < BT) {
    a.best_cut[(size_t)g * B + c0 + tid] = s_best[tid];
    a.best_step[(size_t)g * B + c0 + tid] = s_bstep[tid];
  }
  if (ever) {
    // best_bits: byte (c0 + c) / 8 of each row; tiles of 8 or more columns own whole bytes,
    // narrower ones share bytes with other workgroups and merge through word atomics
    for (int i = tid; i < nr; i += kRThreads) {
      uint32_t bits = 0;
#pragma unroll
      for (int c = 0; c < BT; ++c) {
        const int bit = i * BT + c;
        bits |= ((s_bb[bit >> 5] >> (bit & 31)) & 1u) << c;
      }
      const size_t row = (size_t)(r0 + i) * a.NBY;
      if constexpr (BT >= 8) {
#pragma unroll
        for (int q = 0; q < BT / 8; ++q) {
          const uint32_t mq = ((uint32_t)ever >> (8 * q)) & 0xFFu;
          if (mq) {
            uint8_t* p = a.best_bits + row + (c0 >> 3) + q;
            *p = (uint8_t)((*p & ~mq) | ((bits >> (8 * q)) & mq));
          }
        }
      } else {
        const size_t byte = row + (c0 >> 3);
        const int sh = (int)((byte & 3) * 8 + (c0 & 7));
        unsigned int* w = reinterpret_cast<unsigned int*>(a.best_bits + (byte & ~(size_t)3));
        const uint32_t mw = ((uint32_t)ever & ((1u << BT) - 1u)) << sh;
        atomicAnd(w, ~mw);
        atomicOr(w, (bits << sh) & mw);
      }
    }
  }
}

// prepare != 0: raise the kernels' dynamic LDS limit (outside any stream capture); else launch.
template <typename T, int BT>
hipError_t launch_bt(const StepArgs& a, const int4* items, int nitems, int max_rows, int steps, size_t lds, int wm,
                     hipStream_t s, int prepare) {
  auto go = [&](auto kern) {
    if (prepare)
      return hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds);
    hipLaunchKernelGGL(kern, dim3(nitems), dim3(kRThreads), lds, s, a, items, max_rows, steps);
    return hipGetLastError();
  };
  if (wm == 0) return go(k_resident<T, BT, 0>);
  if (wm == 1) return go(k_resident<T, BT, 1>);
  return go(k_resident<T, BT, 2>);
}

hipError_t dispatch_bt(const StepArgs& a, int dtype, int bt, const int4* items, int nitems, int max_rows, int steps,
                       hipStream_t s, int prepare) {
  const size_t lds = resident_lds_bytes(max_rows, bt, dtype);
  const int wm = a.w == nullptr ? 0 : (a.intw ? 1 : 2);
  if (dtype == 0) {
    switch (bt) {
      case 1: return launch_bt<float, 1>(a, items, nitems, max_rows, steps, lds, wm, s, prepare);
      case 2: return launch_bt<float, 2>(a, items, nitems, max_rows, steps, lds, wm, s, prepare);
      case 4: return launch_bt<float, 4>(a, items, nitems, max_rows, steps, lds, wm, s, prepare);
      case 8: return launch_bt<float, 8>(a, items, nitems, max_rows, steps, lds, wm, s, prepare);
      case 16: return launch_bt<float, 16>(a, items, nitems, max_rows, steps, lds, wm, s, prepare);
      default: return hipErrorInvalidValue;
    }
  }
  switch (bt) {
    case 1: return launch_bt<uint16_t, 1>(a, items, nitems, max_rows, steps, lds, wm, s, prepare);
    case 2: return launch_bt<uint16_t, 2>(a, items, nitems, max_rows, steps, lds, wm, s, prepare);
    case 4: return launch_bt<uint16_t, 4>(a, items, nitems, max_rows, steps, lds, wm, s, prepare);
    case 8: return launch_bt<uint16_t, 8>(a, items, nitems, max_rows, steps, lds, wm, s, prepare);
    case 16: return launch_bt<uint16_t, 16>(a, items, nitems, max_rows, steps, lds, wm, s, prepare);
    default: return hipErrorInvalidValue;
  }
}

__global__ void k_advance(DevCtrl* ctrl, int steps) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctrl->t += steps;
    ctrl->cpend = -1;
    ctrl->fpend = -1;
  }
}

}  // namespace

size_t resident_lds_bytes(int max_rows, int bt, int dtype) {
  const size_t es = dtype == 0 ? 4 : 2;
  return 2 * (size_t)max_rows * bt * es + ((size_t)max_rows * bt + 31) / 32 * 4;
}

hipError_t prepare_resident(const StepArgs& a, int dtype, int bt, int max_rows) {
  return dispatch_bt(a, dtype, bt, nullptr, 0, max_rows, 0, nullptr, 1);
}

hipError_t launch_resident(const StepArgs& a, int dtype, int bt, const int4* items, int nitems, int max_rows,
                           int steps, hipStream_t s) {
  if (nitems <= 0 || steps <= 0) return hipSuccess;
  hipError_t e = dispatch_bt(a, dtype, bt, items, nitems, max_rows, steps, s, 0);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, a.ctrl, steps);
  return hipGetLastError();
}

}  // namespace deco
