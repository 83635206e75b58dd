// Resident step kernel: T steps of projected gradient ascent (Sec. 3.1 eq. (6)-(7)) with the
// rounding (eq. (5), or the lifted rule for l = 1), the exact cut (eq. (1)) and the running
// best of Alg. 1 for every scored iterate, in one launch, with each workgroup's share of X held
// in LDS for all T steps.
//
// Columns (initialisations) never interact in a step: column b of X_{t+1} depends only on
// column b of X_t. So a workgroup that owns one graph's rows and a tile of BT columns can run
// every step of those columns by itself: X_t and X_{t+1} of its tile sit in LDS (two
// buffers), the neighbour gathers read LDS, and the cut of each of its columns is a workgroup
// reduction. No workgroup waits for another, so the launch needs no grid barrier and any
// number of workgroups may be in flight. The kernel applies when 2 n_g BT elements of the
// storage type fit the LDS budget (small and medium graphs, unlifted or l = 1).
//
// Work item i: {graph, first row, end row, first column}. The graph's slots are split into
// equal shares, one per thread, read from an interleaved copy of the slot list built once per
// schedule (k_rhead, k_rstream); rows cut by a share boundary are finished by the thread holding
// their own slot, which adds the following threads' partial sums in thread order. The running
// best (cut, step and the sides of the best iterate) stays in LDS and registers during the
// launch and is written back at the end (tiles narrower than a byte of best_bits through
// k_rbest); the trace and the current cut are written per scored step.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "internal.h"

namespace deco {
namespace {

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

// Threads of a resident workgroup: more threads for narrow tiles (each thread walks its share
// of the graph's slots for every column of the tile).
template <int BT>
struct RTeam {
  static constexpr int NT = BT == 1 ? 1024 : (BT == 2 ? 512 : 256);
};

// Spare rows after a graph's rows in each LDS buffer, one per lane of a wave: the closing
// store of a slot that closes no row of this thread lands in its lane's spare row.
constexpr int kSpareRows = 64;

// Best sides of a row for the tile's columns (bit c: column c0 + c).
template <int BT>
struct RSide {
  using type = typename std::conditional<(BT <= 8), uint8_t, uint16_t>::type;
};

// Sides of BT values from their bit patterns: x > 0 (eq. (5)) is bits > 0 as a signed integer;
// x >= 0 (the lifted rule, -0 included) is the complement of -x > 0.
template <int BT, int LF>
__device__ __forceinline__ uint32_t r_sides(const float (&x)[BT]) {
  uint32_t m = 0;
#pragma unroll
  for (int c = 0; c < BT; ++c) {
    const int b = __float_as_int(x[c]);
    const int z = LF ? 1 - min(max(b ^ (int)0x80000000, 0), 1) : min(max(b, 0), 1);
    m |= (uint32_t)z << c;
  }
  return m;
}

// Bitwise select: a where m is all ones, b where m is zero.
__device__ __forceinline__ int r_sel(int m, int a, int b) { return (a & m) | (b & ~m); }
__device__ __forceinline__ float r_self(int m, float a, float b) {
  return __int_as_float(r_sel(m, __float_as_int(a), __float_as_int(b)));
}

// Side of one value: x > 0 (eq. (5)), or x >= 0 under the lifted rule (-0 included).
template <int LF>
__device__ __forceinline__ bool r_side(float x) { return LF ? x >= 0.0f : x > 0.0f; }

// Slot position of local row v of a graph: its own slot follows the v earlier own slots and
// the edges of the earlier rows.
__device__ __forceinline__ int r_pos(const int* rp, int r0, int v) { return rp[r0 + v] - rp[r0] + v; }

// First local row v in [0, nr] whose own slot lies at or after slot position k.
__device__ __forceinline__ int r_first_row_at(const int* rp, int r0, int nr, long long k) {
  int lo = 0, hi = nr;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (r_pos(rp, r0, mid) < k) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// WM: 0 unit weights (int counts), 1 integer weights (int counts), 2 real weights (double).
//
// Work split: the E slots of the item's graph (its own slot, then the neighbours, per row, in
// CSR order) are cut into NT shares of floor(E t / NT) .. floor(E (t + 1) / NT); share t is
// read from an interleaved copy of the slot list (stream), 4 slots per thread per load, so a
// wave's loads are contiguous. A share may start inside a row (its 'head' row, owned by an
// earlier thread): its sums go to LDS for the owner. A row whose own slot lies in share t
// and that continues past it ('tail' row) is finished by thread t after the first barrier,
// adding the partial sums of the following threads in thread order. The cut counts
// w 1{z_v != z_u} are additive, so every thread counts the slots of its share itself.
// LF: the lifted rounding rule; LAP: the Laplacian form of the gradient (a degree term).
template <typename T, int BT, int WM, int LF, bool LAP>
__global__ __launch_bounds__(RTeam<BT>::NT) void k_resident(StepArgs a, const int4* __restrict__ items,
                                                            const int4* __restrict__ rgs, const int* __restrict__ stream,
                                                            const float* __restrict__ wstream, uint8_t* __restrict__ rbest,
                                                            uint8_t* __restrict__ rimp, int max_rows, int steps) {
  constexpr int NT = RTeam<BT>::NT;
  constexpr int NW = NT / 64;
  using S = typename std::conditional<WM == 2, double, int>::type;
  using SB = typename RSide<BT>::type;
  extern __shared__ __align__(16) unsigned char r_smem[];
  __shared__ S s_red[2][NW * BT];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int4 it = items[blockIdx.x];
  const int g = it.x, r0 = it.y, r1 = it.z, c0 = it.w;
  const int nr = r1 - r0;
  const int4 gs = rgs[g];  // {stream offset, slots per thread (multiple of 4), E, first slot}
  const int E = gs.z;
  T* buf0 = reinterpret_cast<T*>(r_smem);
  T* buf1 = buf0 + (size_t)(max_rows + kSpareRows) * BT;
  SB* s_side = reinterpret_cast<SB*>(buf1 + (size_t)(max_rows + kSpareRows) * BT);
  float* s_part = reinterpret_cast<float*>(
      r_smem +
      ((2 * (size_t)(max_rows + kSpareRows) * BT * sizeof(T) + (size_t)max_rows * sizeof(SB) + 15) & ~(size_t)15));
  // byte offset of this lane's spare row in either buffer
  const int spare = (max_rows + lane) * BT * (int)sizeof(T);
  const long long t0 = a.ctrl->t;
  const int every = a.ctrl->score_every;
  const size_t B = (size_t)a.B;

  // this thread's share [lo, hi) and its header (built with the stream): head row, the
  // threads whose shares start inside its last own row, its own rows [ob, oe)
  const int lo = (int)((long long)E * tid / NT), hi = (int)((long long)E * (tid + 1) / NT);
  const int len = hi - lo;
  const int4 hdr = *reinterpret_cast<const int4*>(stream + gs.x + 4 * tid);
  const int head_row = hdr.x, ntail = hdr.y, ob = hdr.z, oe = hdr.w;

  // X_t0 of the tile into buffer 0; running best of the tile's columns
  const T* X0 = reinterpret_cast<const T*>(a.x[t0 & 1]);
  for (int i = tid; i < nr; i += NT) {
    float v[BT];
    RowIO<T, BT>::load(X0 + (size_t)(r0 + i) * B + c0, v);
    RowIO<T, BT>::store(buf0 + (size_t)i * BT, v);
    s_side[i] = 0;
  }
  double best[BT];
  int bstep[BT];
  float ecw[BT], eta[BT];
#pragma unroll
  for (int c = 0; c < BT; ++c) {
    best[c] = a.best_cut[(size_t)g * B + c0 + c];
    bstep[c] = a.best_step[(size_t)g * B + c0 + c];
    eta[c] = a.eta[c0 + c];
    ecw[c] = eta[c] * a.cW;
  }
  uint32_t ever = 0;  // columns improved during this launch (bit c)
  const int* sp = stream + gs.x + 4 * NT + tid * 4;
  const float* wp = WM != 0 ? wstream + gs.x + 4 * NT + tid * 4 : nullptr;
  const size_t sstride = (size_t)NT * 4;
  __syncthreads();

  for (int s = 0; s < steps; ++s) {
    const long long t = t0 + s;
    const bool do_score = (t % every) == 0;
    const T* cur = (s & 1) ? buf1 : buf0;
    T* nxt = (s & 1) ? buf0 : buf1;
    S cnt[BT];
    float acc[BT], xv[BT];
#pragma unroll
    for (int c = 0; c < BT; ++c) {
      cnt[c] = 0;
      acc[c] = 0.0f;
      xv[c] = 0.0f;
    }
    // The open row: byte offset ri in the buffers (the lane's spare row while none of this
    // thread's rows is open), its values xv, sums acc, weighted degree dsum; while it is the
    // share's head row its sums go to hacc.
    // Narrow tiles (one or two columns per thread) keep the flags as per-lane booleans (head),
    // so each select is one vector instruction with its mask in scalar registers, and carry
    // the open row's store address (sa) instead of ri; with float32 storage sa points at the
    // thread's s_part entry while the open row is the head row, so the store that closes the
    // head row writes its sums there (kHeadStore) and no select per slot keeps hacc.
    // Wide tiles keep integer masks (headm all ones while in the head row) and the open
    // row's sides as bits (zv): their selects stay vector bit operations rather than a
    // scalar mask operation per column.
    constexpr bool kNarrow = BT < 4;
    constexpr bool kHeadStore = kNarrow && sizeof(T) == 4;
    bool head = false;
    int headm = 0;
    uint32_t zv = 0;
    int ri = spare;
    float dsum = 0.0f, hacc[BT];
#pragma unroll
    for (int c = 0; c < BT; ++c) hacc[c] = 0.0f;
    unsigned char* nxt_b = reinterpret_cast<unsigned char*>(nxt);
    unsigned char* const spare_b = nxt_b + spare;
    unsigned char* sa = spare_b;
    if (head_row >= 0) {
      ri = head_row * BT * (int)sizeof(T);
      head = true;
      headm = -1;
      sa = kHeadStore ? reinterpret_cast<unsigned char*>(s_part + tid * BT) : nxt_b + ri;
      RowIO<T, BT>::load(cur + (size_t)head_row * BT, xv);
      if constexpr (!kNarrow) zv = r_sides<BT, LF>(xv);
    }
    auto update = [&](float (&y)[BT]) {
#pragma unroll
      for (int c = 0; c < BT; ++c) {
        float x1;
        if constexpr (LAP)
          x1 = fmaf(eta[c], fmaf(a.cD * dsum, xv[c], a.cW * acc[c]), xv[c]);
        else
          x1 = fmaf(ecw[c], acc[c], xv[c]);
        y[c] = __builtin_amdgcn_fmed3f(x1, -1.0f, 1.0f);
      }
    };
    // nxt minus cur in bytes: the store address of a row from the address it was gathered at
    const ptrdiff_t dnc = nxt_b - reinterpret_cast<const unsigned char*>(cur);
    // one slot (lp: the address its value was gathered at), straight-line: an own slot (flag
    // bit) stores the open row's update (to the spare row unless the open row is one of this
    // thread's) and opens row idx; a neighbour slot is summed and counted
    auto slot = [&](int v, float wq, const float (&xu)[BT], const T* lp) {
      const int idx = v & 0x7FFFFFFF;
      if constexpr (kNarrow) {
        const bool own = v < 0;
        float y[BT];
        update(y);
        if constexpr (kHeadStore) {
#pragma unroll
          for (int c = 0; c < BT; ++c) y[c] = head ? acc[c] : y[c];
          RowIO<T, BT>::store(reinterpret_cast<T*>(own ? sa : spare_b), y);
        } else {
          RowIO<T, BT>::store(reinterpret_cast<T*>(own && !head ? sa : spare_b), y);
#pragma unroll
          for (int c = 0; c < BT; ++c) hacc[c] = own && head ? acc[c] : hacc[c];
        }
        head = head && !own;
        if (do_score) {
#pragma unroll
          for (int c = 0; c < BT; ++c) {
            const bool d = r_side<LF>(xu[c]) != r_side<LF>(xv[c]) && !own;
            if (WM == 2)
              cnt[c] += d ? (S)wq : (S)0;
            else if (WM == 1)
              cnt[c] += d ? (S)(int)wq : (S)0;
            else
              cnt[c] += (S)d;
          }
        }
#pragma unroll
        for (int c = 0; c < BT; ++c) {
          const float an = WM == 0 ? acc[c] + xu[c] : fmaf(wq, xu[c], acc[c]);
          acc[c] = own ? 0.0f : an;
          xv[c] = own ? xu[c] : xv[c];
        }
        sa = own ? const_cast<unsigned char*>(reinterpret_cast<const unsigned char*>(lp)) + dnc : sa;
        if constexpr (LAP) dsum = own ? (WM != 0 ? wq : a.dw[r0 + idx]) : dsum;
      } else {
        const int ownm = v >> 31;
        const uint32_t zu = r_sides<BT, LF>(xu);
        // the update costs BT fused multiply-adds, so only waves with a lane on an own slot
        // take it (long rows make those slots rare)
        if (ownm & ~headm) {
          float y[BT];
          update(y);
          RowIO<T, BT>::store(reinterpret_cast<T*>(nxt_b + ri), y);
        }
#pragma unroll
        for (int c = 0; c < BT; ++c) hacc[c] = r_self(ownm & headm, acc[c], hacc[c]);
        headm &= ~ownm;
        if (do_score) {
          const uint32_t d = (zu ^ zv) & ~(uint32_t)ownm;
#pragma unroll
          for (int c = 0; c < BT; ++c) {
            const int bit = (int)((d >> c) & 1u);
            if (WM == 2)
              cnt[c] += bit ? (S)wq : (S)0;
            else if (WM == 1)
              cnt[c] += (S)((int)wq & -bit);
            else
              cnt[c] += bit;
          }
        }
#pragma unroll
        for (int c = 0; c < BT; ++c) {
          const float an = WM == 0 ? acc[c] + xu[c] : fmaf(wq, xu[c], acc[c]);
          acc[c] = __int_as_float(__float_as_int(an) & ~ownm);
          xv[c] = r_self(ownm, xu[c], xv[c]);
        }
        zv = (uint32_t)r_sel(ownm, (int)zu, (int)zv);
        ri = r_sel(ownm, idx * BT * (int)sizeof(T), ri);
        if constexpr (LAP) dsum = r_self(ownm, WM != 0 ? wq : a.dw[r0 + idx], dsum);
      }
    };
    // slots four at a time from the interleaved stream (the next four in flight); whole
    // batches without predicates, then the share's last partial batch
    const int full = len & ~3;
    int4 sv_next = make_int4(0, 0, 0, 0);
    float4 wv_next = make_float4(1.0f, 1.0f, 1.0f, 1.0f);
    if (len > 0) {
      sv_next = *reinterpret_cast<const int4*>(sp);
      if constexpr (WM != 0) wv_next = *reinterpret_cast<const float4*>(wp);
    }
    for (int jb = 0; jb < len; jb += 4) {
      const int4 sv = sv_next;
      const float4 wv4 = wv_next;
      if (jb + 4 < len) {
        sv_next = *reinterpret_cast<const int4*>(sp + (size_t)((jb >> 2) + 1) * sstride);
        if constexpr (WM != 0) wv_next = *reinterpret_cast<const float4*>(wp + (size_t)((jb >> 2) + 1) * sstride);
      }
      const int sl[4] = {sv.x, sv.y, sv.z, sv.w};
      const float wl[4] = {wv4.x, wv4.y, wv4.z, wv4.w};
      float xb[4][BT];
      const T* lp[4];
      if (jb < full) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          lp[q] = cur + (size_t)(sl[q] & 0x7FFFFFFF) * BT;
          RowIO<T, BT>::load(lp[q], xb[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) slot(sl[q], wl[q], xb[q], lp[q]);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          lp[q] = cur + (size_t)(jb + q < len ? sl[q] & 0x7FFFFFFF : 0) * BT;
          RowIO<T, BT>::load(lp[q], xb[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (jb + q < len) slot(sl[q], wl[q], xb[q], lp[q]);
      }
    }
    // the head row's sums for its owner (zeros when the share has no head row)
    const bool in_head = kNarrow ? head : headm != 0;
    if constexpr (kNarrow) {
      if (!in_head) ri = (int)(sa - nxt_b);
    }
    if constexpr (kHeadStore) {
      // a head row closed inside the share has stored its sums already
      if (in_head || head_row < 0)
#pragma unroll
        for (int c = 0; c < BT; ++c) s_part[tid * BT + c] = in_head ? acc[c] : 0.0f;
    } else {
#pragma unroll
      for (int c = 0; c < BT; ++c) s_part[tid * BT + c] = in_head ? acc[c] : hacc[c];
    }
    const bool open_own = !in_head && ri != spare;
    const bool tail = open_own && ntail > 0;
    if (open_own && ntail == 0) {
      float y[BT];
      update(y);
      RowIO<T, BT>::store(reinterpret_cast<T*>(nxt_b + ri), y);
    }
    if (do_score) {
#pragma unroll
      for (int c = 0; c < BT; ++c) {
        S v = cnt[c];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) s_red[s & 1][wv * BT + c] = v;
      }
    }
    __syncthreads();  // head sums and wave counts are in LDS
    if (tail) {
      for (int k = 1; k <= ntail; ++k)
#pragma unroll
        for (int c = 0; c < BT; ++c) acc[c] += s_part[(tid + k) * BT + c];
      float y[BT];
      update(y);
      RowIO<T, BT>::store(reinterpret_cast<T*>(nxt_b + ri), y);
    }
    __syncthreads();  // X_t+1 complete
    if (do_score) {
      uint32_t m = 0;
#pragma unroll
      for (int c = 0; c < BT; ++c) {
        S tot = 0;
#pragma unroll
        for (int q = 0; q < NW; ++q) tot += s_red[s & 1][q * BT + c];
        const double cut = 0.5 * (double)tot;
        if (tid == c) {
          const size_t idx = (size_t)g * B + c0 + c;
          a.cur_cut[idx] = cut;
          if (a.trace) a.trace[(size_t)(t % a.trace_cap) * a.G * B + idx] = cut;
        }
        if (cut > best[c]) {
          best[c] = cut;
          bstep[c] = (int)t;
          m |= 1u << c;
        }
      }
      ever |= m;
      if (m) {
        // sides of X_t (buffer cur) of this thread's own rows for the improved columns;
        // the next step rewrites those rows only after this
        for (int i = ob; i < oe; ++i) {
          float x[BT];
          RowIO<T, BT>::load(cur + (size_t)i * BT, x);
          const uint32_t z = r_sides<BT, LF>(x);
          s_side[i] = (SB)((s_side[i] & ~m) | (z & m));
        }
      }
    }
  }
  __syncthreads();

  // X_{t0 + steps} back to global memory; running best and its sides
  const T* fin = (steps & 1) ? buf1 : buf0;
  T* Xo = reinterpret_cast<T*>(a.x[(t0 + steps) & 1]);
  for (int i = tid; i < nr; i += NT) {
    float v[BT];
    RowIO<T, BT>::load(fin + (size_t)i * BT, v);
    RowIO<T, BT>::store(Xo + (size_t)(r0 + i) * B + c0, v);
  }
  if (tid < BT) {
#pragma unroll
    for (int c = 0; c < BT; ++c)
      if (c == tid) {
        a.best_cut[(size_t)g * B + c0 + c] = best[c];
        a.best_step[(size_t)g * B + c0 + c] = bstep[c];
      }
  }
  if constexpr (BT >= 8) {
    // best_bits: tiles of 8 or more columns own whole bytes of each row
    if (ever) {
      for (int i = tid; i < nr; i += NT) {
        const uint32_t bits = s_side[i];
        const size_t rowb = (size_t)(r0 + i) * a.NBY;
#pragma unroll
        for (int q = 0; q < BT / 8; ++q) {
          const uint32_t mq = (ever >> (8 * q)) & 0xFFu;
          if (mq) {
            uint8_t* p = a.best_bits + rowb + (c0 >> 3) + q;
            *p = (uint8_t)((*p & ~mq) | ((bits >> (8 * q)) & mq));
          }
        }
      }
    }
  } else {
    // narrower tiles share bytes of best_bits with other workgroups: the sides go to the
    // tile's own byte array (rows in order) and the improved columns to a flag byte, which
    // k_rbest merges after the launch
    const int tile = c0 / BT;
    if (tid == 0) rimp[(size_t)g * (B / BT) + tile] = (uint8_t)ever;
    if (ever)
      for (int i = tid; i < nr; i += NT) rbest[(size_t)tile * a.n + r0 + i] = (uint8_t)s_side[i];
  }
}

// Merge of the narrow resident tiles' best sides into best_bits: byte k of row r takes, for
// each tile of the byte's columns improved during the launch, that tile's bits.
template <int BT>
__global__ void k_rbest(StepArgs a, const uint8_t* __restrict__ rbest, const uint8_t* __restrict__ rimp,
                        const int* __restrict__ goff) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n * a.NBY) return;
  const long long r = i / a.NBY;
  const int k = (int)(i % a.NBY);
  int lo = 0, hi = a.G - 1;  // graph of row r
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (goff[mid] <= r) lo = mid; else hi = mid - 1;
  }
  const int ntile = a.B / BT;
  uint32_t byte = a.best_bits[i];
  const uint32_t old = byte;
#pragma unroll
  for (int q = 0; q < 8 / BT; ++q) {
    const int t = k * (8 / BT) + q;
    if (t < ntile) {
      const uint32_t m = rimp[(size_t)lo * ntile + t];
      if (m) {
        const uint32_t bits = rbest[(size_t)t * a.n + r];
        byte = (byte & ~(m << (q * BT))) | ((bits & m) << (q * BT));
      }
    }
  }
  if (byte != old) a.best_bits[i] = (uint8_t)byte;
}

// Headers of the resident schedule's shares: for thread t of graph g (share [lo, hi) of the
// graph's E slots) {head row (the row holding slot lo when that is not its own slot, else
// -1), the number of following threads whose shares start inside its last own row when that
// row continues past hi, first own row, end of its own rows} at stream[off_g + 4 t].
__global__ void k_rhead(int G, int nt, const int4* __restrict__ rgs, const int* __restrict__ goff,
                        const int* __restrict__ rp, int* __restrict__ stream) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)G * nt) return;
  const int g = (int)(i / nt), t = (int)(i % nt);
  const int4 gs = rgs[g];
  const int r0 = goff[g], nr = goff[g + 1] - r0;
  const long long E = gs.z;
  const int lo = (int)(E * t / nt), hi = (int)(E * (t + 1) / nt);
  const int ob = r_first_row_at(rp, r0, nr, lo);
  const int oe = r_first_row_at(rp, r0, nr, hi);
  const int head_row = (lo < E && (ob >= nr || r_pos(rp, r0, ob) != lo)) ? ob - 1 : -1;
  int ntail = 0;
  if (oe > ob) {
    const long long row_end = r_pos(rp, r0, oe);  // end of the last own row
    if (row_end > hi) ntail = (int)((row_end * nt + E - 1) / E) - t - 1;
  }
  reinterpret_cast<int4*>(stream + gs.x)[t] = make_int4(head_row, ntail, ob, oe);
}

// Interleaved slot streams of the resident schedule: after the headers, slot j of thread t's
// share of graph g (slot floor(E t / NT) + j of the graph) at
// stream[off_g + 4 NT + (j / 4) NT 4 + 4 t + j % 4], as a local row index (own slots keep the
// flag bit), with its weight beside it.
__global__ void k_rstream(long long nslots, int G, int nt, const int4* __restrict__ rgs, const int* __restrict__ goff,
                          const int* __restrict__ slots, const float* __restrict__ sw, int* __restrict__ stream,
                          float* __restrict__ wstream) {
  const long long K = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= nslots) return;
  int lo = 0, hi = G - 1;  // last graph whose first slot is <= K
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (rgs[mid].w <= K) lo = mid; else hi = mid - 1;
  }
  const int4 gs = rgs[lo];
  const long long E = gs.z, k = K - gs.w;
  const long long t = ((k + 1) * nt - 1) / E;
  const long long j = k - E * t / nt;
  const size_t dst = (size_t)gs.x + (size_t)nt * 4 + (size_t)(j >> 2) * nt * 4 + (size_t)t * 4 + (size_t)(j & 3);
  const int v = slots[K];
  const int r0 = goff[lo];
  stream[dst] = v < 0 ? (int)(0x80000000u | (unsigned)((v & 0x7FFFFFFF) - r0)) : v - r0;
  if (wstream) wstream[dst] = sw[K];
}

// prepare != 0: raise the kernels' dynamic LDS limit (outside any stream capture); else launch.
template <typename T, int BT>
hipError_t launch_bt(const StepArgs& a, const int4* items, int nitems, const int4* rgs, const int* stream,
                     const float* wstream, uint8_t* rbest, uint8_t* rimp, const int* goff, int max_rows, int steps,
                     size_t lds, int wm, hipStream_t s, int prepare) {
  auto go = [&](auto kern) {
    if (prepare)
      return hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds);
    hipLaunchKernelGGL(kern, dim3(nitems), dim3(RTeam<BT>::NT), lds, s, a, items, rgs, stream, wstream, rbest, rimp,
                       max_rows, steps);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && BT < 8) {
      const long long work = a.n * a.NBY;
      hipLaunchKernelGGL(k_rbest<BT < 8 ? BT : 1>, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, a, rbest,
                         rimp, goff);
      e = hipGetLastError();
    }
    return e;
  };
  auto by_form = [&](auto lf) {
    constexpr int LF = decltype(lf)::value;
    if (a.cD != 0.0f) {
      if (wm == 0) return go(k_resident<T, BT, 0, LF, true>);
      if (wm == 1) return go(k_resident<T, BT, 1, LF, true>);
      return go(k_resident<T, BT, 2, LF, true>);
    }
    if (wm == 0) return go(k_resident<T, BT, 0, LF, false>);
    if (wm == 1) return go(k_resident<T, BT, 1, LF, false>);
    return go(k_resident<T, BT, 2, LF, false>);
  };
  return a.lifted ? by_form(std::integral_constant<int, 1>{}) : by_form(std::integral_constant<int, 0>{});
}

hipError_t dispatch_bt(const StepArgs& a, int dtype, int bt, const int4* items, int nitems, const int4* rgs,
                       const int* stream, const float* wstream, uint8_t* rbest, uint8_t* rimp, const int* goff,
                       int max_rows, int steps, hipStream_t s, int prepare) {
  const size_t lds = resident_lds_bytes(max_rows, bt, dtype);
  const int wm = a.w == nullptr ? 0 : (a.intw ? 1 : 2);
  if (dtype == 0) {
    switch (bt) {
      case 1: return launch_bt<float, 1>(a, items, nitems, rgs, stream, wstream, rbest, rimp, goff, max_rows, steps, lds, wm, s, prepare);
      case 2: return launch_bt<float, 2>(a, items, nitems, rgs, stream, wstream, rbest, rimp, goff, max_rows, steps, lds, wm, s, prepare);
      case 4: return launch_bt<float, 4>(a, items, nitems, rgs, stream, wstream, rbest, rimp, goff, max_rows, steps, lds, wm, s, prepare);
      case 8: return launch_bt<float, 8>(a, items, nitems, rgs, stream, wstream, rbest, rimp, goff, max_rows, steps, lds, wm, s, prepare);
      case 16: return launch_bt<float, 16>(a, items, nitems, rgs, stream, wstream, rbest, rimp, goff, max_rows, steps, lds, wm, s, prepare);
      default: return hipErrorInvalidValue;
    }
  }
  switch (bt) {
    case 1: return launch_bt<uint16_t, 1>(a, items, nitems, rgs, stream, wstream, rbest, rimp, goff, max_rows, steps, lds, wm, s, prepare);
    case 2: return launch_bt<uint16_t, 2>(a, items, nitems, rgs, stream, wstream, rbest, rimp, goff, max_rows, steps, lds, wm, s, prepare);
    case 4: return launch_bt<uint16_t, 4>(a, items, nitems, rgs, stream, wstream, rbest, rimp, goff, max_rows, steps, lds, wm, s, prepare);
    case 8: return launch_bt<uint16_t, 8>(a, items, nitems, rgs, stream, wstream, rbest, rimp, goff, max_rows, steps, lds, wm, s, prepare);
    case 16: return launch_bt<uint16_t, 16>(a, items, nitems, rgs, stream, wstream, rbest, rimp, goff, max_rows, steps, lds, wm, s, prepare);
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

int resident_threads(int bt) {
  return bt == 1 ? RTeam<1>::NT : (bt == 2 ? RTeam<2>::NT : RTeam<4>::NT);
}

size_t resident_lds_bytes(int max_rows, int bt, int dtype) {
  const size_t es = dtype == 0 ? 4 : 2;
  const size_t side = bt <= 8 ? 1 : 2;
  const size_t front = (2 * (size_t)(max_rows + kSpareRows) * bt * es + (size_t)max_rows * side + 15) & ~(size_t)15;
  return front + (size_t)resident_threads(bt) * bt * sizeof(float);
}

hipError_t prepare_resident(const StepArgs& a, int dtype, int bt, int max_rows) {
  return dispatch_bt(a, dtype, bt, nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, max_rows, 0, nullptr,
                     1);
}

hipError_t build_resident_stream(long long nslots, int G, int bt, const int4* rgs, const int* goff, const int* rp,
                                 const int* slots, const float* sw, int* stream, float* wstream, hipStream_t s) {
  if (nslots <= 0) return hipSuccess;
  const int threads = 256, nt = resident_threads(bt);
  const long long hblocks = ((long long)G * nt + threads - 1) / threads;
  hipLaunchKernelGGL(k_rhead, dim3((unsigned)hblocks), dim3(threads), 0, s, G, nt, rgs, goff, rp, stream);
  const long long blocks = (nslots + threads - 1) / threads;
  hipLaunchKernelGGL(k_rstream, dim3((unsigned)blocks), dim3(threads), 0, s, nslots, G, nt, rgs, goff, slots, sw,
                     stream, wstream);
  return hipGetLastError();
}

hipError_t launch_resident(const StepArgs& a, int dtype, int bt, const int4* items, int nitems, const int4* rgs,
                           const int* stream, const float* wstream, uint8_t* rbest, uint8_t* rimp, const int* goff,
                           int max_rows, int steps, hipStream_t s) {
  if (nitems <= 0 || steps <= 0) return hipSuccess;
  hipError_t e = dispatch_bt(a, dtype, bt, items, nitems, rgs, stream, wstream, rbest, rimp, goff, max_rows, steps, s, 0);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, a.ctrl, steps);
  return hipGetLastError();
}

}  // namespace deco
