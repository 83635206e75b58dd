// Device kernels of the DECO library for gfx950 (CDNA4, wave64).
//
// The hot kernel, k_step, performs one step of batched projected gradient ascent
// (Sec. 3.1 eq. (6)-(7), Sec. 3.2 lifted update) fused with the exact scoring of the
// iterate it reads (eq. (5) / lifted rounding, eq. (1)) and the running best of Alg. 1-2:
//
//   for every row v and initialisation b (all l components):
//     acc   = sum_{u in N(v)} w_vu X_t[u, i, b]           (float32)
//     X_t+1 = clip(X_t[v] + eta_b (cW acc + cD d_w(v) X_t[v]), -1, 1)
//     score += w_vu 1{z_t(v) != z_t(u)}                   (double, exact for integer w)
//
// Mapping. X is node-major: row v holds its l*B values contiguously. One initialisation
// tile of a row (Bt = Wc*VEC columns, at most 256, for every component) is held by a row
// team of Wc lanes with 16-byte loads (8-byte for lifted rows, or 4-byte bfloat16 pairs); a
// 256-thread workgroup has NS = 256/Wc teams. The graph is read through
// its slot list: row v is its own index (top bit set) followed by its neighbours, so a team
// walks a flat stream of slots and never waits on a row boundary. Work items are row ranges
// of one graph and one tile, grouped per XCD (workgroup i runs on XCD i % 8) and walked by a
// persistent grid:
//  * a normal item (rows of degree <= the long-row threshold, at most kEmax slots and
//    kRmax rows) copies its slots (and slot weights) into LDS with coalesced loads; team s
//    takes the rows whose own slot lies in the s-th equal share of the item's slots and
//    walks them in windows of W slots: all W gathers (own rows and neighbours alike) are
//    issued before any is used, then folded in order, a self slot closing the previous
//    row (update, store, cut bits) and opening its own;
//  * a long-row item holds one row: every team takes a contiguous share of each staged
//    chunk of its neighbour slots, and the float32 partial sums are reduced in a fixed
//    order (butterfly inside a wave, then the waves in order through LDS) before team 0
//    finishes the row.
// Score partials stay in registers (int32 for integer weights, exact; float otherwise)
// until the item ends; then a wave reduction and an LDS reduction in double and one double
// atomic per initialisation into one of R replicated accumulators. After its rows, an item
// folds the previous scored step's improved cut bits into best_bits for its rows and tile.
// Completion uses a two-level ticket (per XCD, then global) so no address takes more than
// one atomic per workgroup of one XCD. The last workgroup turns the sums into cuts,
// updates best / best step / improvement mask and advances the step counter.
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

// Raw 16-byte (or scalar) loads kept packed while in flight, unpacked to float at use.
template <typename T, int VEC>
struct VecIO;

template <>
struct VecIO<float, 4> {
  using raw = float4;
  static __device__ __forceinline__ raw load_raw(const float* p) { return *reinterpret_cast<const float4*>(p); }
  static __device__ __forceinline__ raw zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
  static __device__ __forceinline__ void unpack(const raw& v, float (&o)[4]) {
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
struct VecIO<float, 2> {
  using raw = float2;
  static __device__ __forceinline__ raw load_raw(const float* p) { return *reinterpret_cast<const float2*>(p); }
  static __device__ __forceinline__ raw zero() { return make_float2(0.f, 0.f); }
  static __device__ __forceinline__ void unpack(const raw& v, float (&o)[2]) {
    o[0] = v.x;
    o[1] = v.y;
  }
  static __device__ __forceinline__ void store(float* p, const float (&o)[2]) {
    *reinterpret_cast<float2*>(p) = make_float2(o[0], o[1]);
  }
};

template <>
struct VecIO<float, 1> {
  using raw = float;
  static __device__ __forceinline__ raw load_raw(const float* p) { return *p; }
  static __device__ __forceinline__ raw zero() { return 0.f; }
  static __device__ __forceinline__ void unpack(const raw& v, float (&o)[1]) { o[0] = v; }
  static __device__ __forceinline__ void store(float* p, const float (&o)[1]) { *p = o[0]; }
};

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two float32 -> a packed pair of bfloat16 (hardware conversion, round to nearest even).
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2{lo, hi}), bf16x2));
}

template <>
struct VecIO<uint16_t, 8> {
  using raw = uint4;
  static __device__ __forceinline__ raw load_raw(const uint16_t* p) { return *reinterpret_cast<const uint4*>(p); }
  static __device__ __forceinline__ raw zero() { return make_uint4(0u, 0u, 0u, 0u); }
  static __device__ __forceinline__ void unpack(const raw& v, float (&o)[8]) {
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
    v.x = pack_bf16(o[0], o[1]);
    v.y = pack_bf16(o[2], o[3]);
    v.z = pack_bf16(o[4], o[5]);
    v.w = pack_bf16(o[6], o[7]);
    *reinterpret_cast<uint4*>(p) = v;
  }
};

template <>
struct VecIO<uint16_t, 4> {
  using raw = uint2;
  static __device__ __forceinline__ raw load_raw(const uint16_t* p) { return *reinterpret_cast<const uint2*>(p); }
  static __device__ __forceinline__ raw zero() { return make_uint2(0u, 0u); }
  static __device__ __forceinline__ void unpack(const raw& v, float (&o)[4]) {
    o[0] = bf2f(v.x & 0xFFFFu);
    o[1] = bf2f(v.x >> 16);
    o[2] = bf2f(v.y & 0xFFFFu);
    o[3] = bf2f(v.y >> 16);
  }
  static __device__ __forceinline__ void store(uint16_t* p, const float (&o)[4]) {
    uint2 v;
    v.x = pack_bf16(o[0], o[1]);
    v.y = pack_bf16(o[2], o[3]);
    *reinterpret_cast<uint2*>(p) = v;
  }
};

template <>
struct VecIO<uint16_t, 2> {
  using raw = uint32_t;
  static __device__ __forceinline__ raw load_raw(const uint16_t* p) { return *reinterpret_cast<const uint32_t*>(p); }
  static __device__ __forceinline__ raw zero() { return 0u; }
  static __device__ __forceinline__ void unpack(const raw& v, float (&o)[2]) {
    o[0] = bf2f(v & 0xFFFFu);
    o[1] = bf2f(v >> 16);
  }
  static __device__ __forceinline__ void store(uint16_t* p, const float (&o)[2]) {
    *reinterpret_cast<uint32_t*>(p) = pack_bf16(o[0], o[1]);
  }
};

// The 32-bit words (bfloat16 pairs) of a raw bfloat16 load.
__device__ __forceinline__ void raw_words(const uint4& v, uint32_t (&w)[4]) {
  w[0] = v.x;
  w[1] = v.y;
  w[2] = v.z;
  w[3] = v.w;
}
__device__ __forceinline__ void raw_words(const uint2& v, uint32_t (&w)[2]) {
  w[0] = v.x;
  w[1] = v.y;
}
__device__ __forceinline__ void raw_words(const uint32_t& v, uint32_t (&w)[1]) { w[0] = v; }

template <>
struct VecIO<uint16_t, 1> {
  using raw = uint32_t;
  static __device__ __forceinline__ raw load_raw(const uint16_t* p) { return *p; }
  static __device__ __forceinline__ raw zero() { return 0u; }
  static __device__ __forceinline__ void unpack(const raw& v, float (&o)[1]) { o[0] = bf2f(v); }
  static __device__ __forceinline__ void store(uint16_t* p, const float (&o)[1]) {
    *p = (uint16_t)(pack_bf16(o[0], 0.0f) & 0xFFFFu);
  }
};

// Side of one initialisation from its l component values (float32, order i = 0..l-1).
// The sum starts from x[0] itself: 0 + x[0] differs from x[0] only for x[0] = -0, and no
// later sum or the comparison with 0 tells -0 from +0.
template <int L>
__device__ __forceinline__ bool side_of(const float (&x)[L], int lifted) {
  float s = x[0];
#pragma unroll
  for (int i = 1; i < L; ++i) s = s + x[i];
  if constexpr (L > 1) {
    return s >= 0.0f;  // l > 1 only exists lifted
  } else {
    const bool pos = x[0] > 0.0f, nonneg = s >= 0.0f;  // both formed, then selected (no branch)
    return lifted ? nonneg : pos;
  }
}

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kSlotPad = 32;  // staged slots are read up to a window past a share

// Slots gathered together by one row team: 16 loads in flight per lane for unlifted rows
// (12 for 16-byte lanes, whose values take twice the registers), 8 when the l > 1
// components also hold registers (32 for one-element lanes), divided among the l
// components.
template <typename T, int L, int VEC>
struct Tune {
  static constexpr int kLoads = VEC == 1 ? 32 : (L == 1 ? ((int)sizeof(T) * VEC >= 16 ? 12 : 16) : 8);
  static constexpr int W = kLoads / L < 1 ? 1 : kLoads / L;
};

// Weight modes: unit weights (no weight loads), weights of +-1, integer weights of
// magnitude <= 1024 (int32 score partials, exact), real weights (float32 score partials).
enum : int { kUnitW = 0, kIntW = 1, kRealW = 2, kPm1W = 3 };
template <int WM>
struct ScoreType {
  using type = int;
};
template <>
struct ScoreType<kRealW> {
  using type = float;
};

typedef short i16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Per 16-bit lane of a word of two bfloat16: 1 where the value is <= 0 (+0, -0 and
// negatives), else 0. The saturating decrement leaves the sign bit set exactly for those
// raw values (-0 = 0x8000 saturates at itself).
__device__ __forceinline__ i16x2 nonpos_pair(uint32_t word) {
  const i16x2 d = __builtin_elementwise_sub_sat(__builtin_bit_cast(i16x2, word), (i16x2){1, 1});
  return __builtin_bit_cast(i16x2, __builtin_bit_cast(u16x2, d) >> (u16x2){15, 15});
}

// acc + (the low or high bfloat16 of word) * (the matching half of wpair), in float32.
// wpair must be a register value: the compiler may encode a constant pair as an inline
// float constant, which this instruction does not read as a bfloat16 pair.
__device__ __forceinline__ float dot2_bf16(uint32_t word, uint32_t wpair, float acc) {
  return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, word), __builtin_bit_cast(bf16x2, wpair), acc,
                                         false);
}

// Sides of the VEC initialisations of one lane as a bit mask.
template <int L, int VEC>
__device__ __forceinline__ uint32_t side_mask(const float (&x)[L][VEC], int lifted) {
  uint32_t m = 0;
#pragma unroll
  for (int e = 0; e < VEC; ++e) {
    float g[L];
#pragma unroll
    for (int i = 0; i < L; ++i) g[i] = x[i][e];
    m |= (side_of<L>(g, lifted) ? 1u : 0u) << e;
  }
  return m;
}

// Sides of the VEC initialisations of one lane from its l raw component vectors.
template <typename T, int VEC, int L>
__device__ __forceinline__ uint32_t side_mask_raw(const typename VecIO<T, VEC>::raw (&xr)[L], int lifted) {
  float x[L][VEC];
#pragma unroll
  for (int i = 0; i < L; ++i) VecIO<T, VEC>::unpack(xr[i], x[i]);
  return side_mask<L, VEC>(x, lifted);
}

// Score counters of unlifted bfloat16 rows with unit or +-1 weights stay in packed 16-bit
// pairs (one pair per 32-bit word of the row).
template <typename T, int L, int VEC, int WM>
struct Packed {
  static constexpr bool value = sizeof(T) == 2 && L == 1 && VEC >= 2 && (WM == kUnitW || WM == kPm1W);
};

// The open row of a team: its own values (storage format), the running neighbour sums, its
// sides, and the score counters of the neighbours taken so far: wsum = sum of w and
// zs = sum of w z_u per initialisation (z_u the neighbour's side), from which the cut
// contribution sum_u w 1{z_u != z_v} = z_v ? wsum - zs : zs follows when the row closes. A
// 'head' row is the continuation of a row whose own slot lies in an earlier team's share:
// its sums go to that team.
template <typename T, int L, int VEC, int WM>
struct RowState {
  using ST = typename ScoreType<WM>::type;
  static constexpr bool kPacked = Packed<T, L, VEC, WM>::value;
  typename VecIO<T, VEC>::raw xv[L];
  float acc[L][VEC];
  i16x2 zp[kPacked ? VEC / 2 : 1];
  ST zs[kPacked ? 1 : VEC];
  ST wsum;   // weights: accumulated per slot; unit weights: set from positions before use
  int open;  // staged position of the first slot of the open row taken in this share
  uint32_t zm;
  int row;    // -1 while no row is open
  float dsum; // weighted degree (Laplacian form)
  bool head;  // continuation of an earlier team's row
  bool lazy;  // zm not yet formed from xv
  uint32_t ulo, uhi;  // bfloat16 pairs (1, 0) and (0, 1) for the dot instruction (unit weights)
  __device__ __forceinline__ void set_unit_pairs() {
    ulo = 0x00003F80u;
    asm volatile("" : "+v"(ulo));  // keep the pair in a register, formed once
    uhi = ulo << 16;
    asm volatile("" : "+v"(uhi));
  }
};

// Score partials of a workgroup's current item per initialisation of the lane: packed 16-bit
// pairs for the packed rows (at most kEmax slots, each adding at most 1 in magnitude, are
// taken before a flush), int32 (integer weights) or float32 (real weights) otherwise.
template <typename T, int L, int VEC, int WM>
struct ScoreAcc {
  using ST = typename ScoreType<WM>::type;
  static constexpr bool kPacked = Packed<T, L, VEC, WM>::value;
  i16x2 p[kPacked ? VEC / 2 : 1];
  ST s[kPacked ? 1 : VEC];
  __device__ __forceinline__ void clear() {
    if constexpr (kPacked) {
#pragma unroll
      for (int k = 0; k < VEC / 2; ++k) p[k] = i16x2{0, 0};
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e) s[e] = 0;
    }
  }
  __device__ __forceinline__ double get(int e) const {
    if constexpr (kPacked)
      return (double)((e & 1) ? p[e >> 1].y : p[e >> 1].x);
    else
      return (double)s[e];
  }
};

template <typename T, int L, int VEC, int WM>
__device__ __forceinline__ void reset_counters(RowState<T, L, VEC, WM>& st) {
  if constexpr (RowState<T, L, VEC, WM>::kPacked) {
#pragma unroll
    for (int k = 0; k < VEC / 2; ++k) st.zp[k] = i16x2{0, 0};
  } else {
#pragma unroll
    for (int e = 0; e < VEC; ++e) st.zs[e] = 0;
  }
  st.wsum = 0;
}

// Adds the cut contribution of the neighbours counted in st to sc and clears the counters.
// Packed counters hold sum w 1{x' <= 0} with x' = x_u unlifted (so sum w z_u = wsum minus
// the counter) and x' = -x_u lifted (the counter itself, see take_slot); then
// d = z + z_v (wsum - 2 z) per 16-bit lane.
template <typename T, int L, int VEC, int WM>
__device__ __forceinline__ void close_score(RowState<T, L, VEC, WM>& st, ScoreAcc<T, L, VEC, WM>& sc, int lifted) {
  using ST = typename ScoreType<WM>::type;
  if constexpr (RowState<T, L, VEC, WM>::kPacked) {
    const i16x2 w2 = {(short)st.wsum, (short)st.wsum};
    const i16x2 zz = __builtin_bit_cast(i16x2, st.zm | (st.zm << 16));
#pragma unroll
    for (int k = 0; k < VEC / 2; ++k) {
      const i16x2 zv = (zz >> i16x2{(short)(2 * k), (short)(2 * k + 1)}) & i16x2{1, 1};
      const i16x2 z = lifted ? st.zp[k] : w2 - st.zp[k];
      sc.p[k] += z + zv * (w2 - z - z);
    }
  } else {
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const ST z = st.zs[e];
      sc.s[e] += ((st.zm >> e) & 1u) ? st.wsum - z : z;
    }
  }
  reset_counters(st);
}

// A team's partial sums of its head row, for the team that owns the row.
template <int L, int VEC>
__device__ __forceinline__ void put_part(float* s_part, int idx, const float (&acc)[L][VEC]) {
#pragma unroll
  for (int i = 0; i < L; ++i)
#pragma unroll
    for (int e = 0; e < VEC; ++e) s_part[idx + i * VEC + e] = acc[i][e];
}

// Projected update of one row and its cut bits for the lanes' initialisations. Every lane
// of the team calls it (the bit byte is assembled with shuffles inside the team); 'lead'
// lanes store.
// eta points at the tile's step sizes in LDS: eta[e] = eta_b, eta[256 + e] = eta_b * cW. In
// the cut form x + eta (cW acc) is formed as one fused multiply-add with the exact product
// (eta cW) acc (cW is -1/2 or -1).
template <typename T, int VEC, int L, int WM>
__device__ __forceinline__ void finish_row(const StepArgs& a, T* __restrict__ Y, uint8_t* __restrict__ bw,
                                           bool do_score, bool lead, int bl, int lc, int gb,
                                           const float* __restrict__ eta, const RowState<T, L, VEC, WM>& st,
                                           float* vel) {
  if (a.do_update && lead) {
#pragma unroll
    for (int i = 0; i < L; ++i) {
      float xv[VEC], y[VEC];
      VecIO<T, VEC>::unpack(st.xv[i], xv);
      if (vel == nullptr) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          float v;
          if (a.cD != 0.0f)
            v = fmaf(eta[e], fmaf(a.cD * st.dsum, xv[e], a.cW * st.acc[i][e]), xv[e]);
          else
            v = fmaf(eta[256 + e], st.acc[i][e], xv[e]);
          y[e] = __builtin_amdgcn_fmed3f(v, -1.0f, 1.0f);
        }
      } else {
        // heavy-ball momentum: V' = mu V + G, X' = clip(X + eta V'), V in float32 beside X
        float* vp = vel + (size_t)st.row * a.C + (size_t)i * a.B + bl;
        float vo[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) vo[e] = vp[e];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const float g =
              a.cD != 0.0f ? fmaf(a.cD * st.dsum, xv[e], a.cW * st.acc[i][e]) : a.cW * st.acc[i][e];
          const float vn = fmaf(a.mu, vo[e], g);
          vo[e] = vn;
          y[e] = __builtin_amdgcn_fmed3f(fmaf(eta[e], vn, xv[e]), -1.0f, 1.0f);
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) vp[e] = vo[e];
      }
      VecIO<T, VEC>::store(Y + (size_t)st.row * a.C + (size_t)i * a.B + bl, y);
    }
  }
  // cut bits of X_t: one byte per 8 initialisations, assembled over gb lanes
  uint32_t byte = (st.zm & ((1u << VEC) - 1u)) << ((lc * VEC) & 7);
  // neighbour lanes 1 and 2 apart through DPP quad permutations, 4 apart through LDS
  if (gb > 1) byte |= (uint32_t)__builtin_amdgcn_mov_dpp((int)byte, 0xB1, 0xF, 0xF, false);  // lanes i ^ 1
  if (gb > 2) byte |= (uint32_t)__builtin_amdgcn_mov_dpp((int)byte, 0x4E, 0xF, 0xF, false);  // lanes i ^ 2
  if (gb > 4) byte |= __shfl_xor(byte, 4);
  if (do_score && lead && (lc % gb) == 0) bw[(size_t)st.row * a.NBY + (bl >> 3)] = (uint8_t)byte;
}

// Closes the open row of a team inside its share: score contribution, then the row's
// partial sums to their owner (head row) or the update of the complete row.
template <typename T, int VEC, int L, int WM>
__device__ __forceinline__ void close_row(const StepArgs& a, T* __restrict__ Y, uint8_t* __restrict__ bw,
                                          float* s_part, int part_idx, bool do_score, int bl, int lc, int gb,
                                          const float* __restrict__ eta, RowState<T, L, VEC, WM>& st,
                                          ScoreAcc<T, L, VEC, WM>& sc, int pos, int lifted, float* vel) {
  if constexpr (WM == kUnitW) st.wsum = pos - st.open;  // neighbours taken in this share
  if (WM == kUnitW && !st.head) st.dsum = (float)st.wsum;  // degree: the row's slots were all taken here
  if (do_score) close_score(st, sc, lifted);
  if (st.head)
    put_part<L, VEC>(s_part, part_idx, st.acc);
  else
    finish_row<T, VEC, L, WM>(a, Y, bw, do_score, true, bl, lc, gb, eta, st, vel);
}

// Opens the row whose own slot was just read.
template <typename T, int L, int VEC, int WM>
__device__ __forceinline__ void open_row(RowState<T, L, VEC, WM>& st, int row,
                                         const typename VecIO<T, VEC>::raw (&xr)[L], float wself, int lifted,
                                         int pos) {
  st.row = row;
  st.open = pos + 1;
  st.head = false;
  st.dsum = WM == kUnitW ? 0.0f : wself;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    st.xv[i] = xr[i];
#pragma unroll
    for (int e = 0; e < VEC; ++e) st.acc[i][e] = 0.0f;
  }
  if constexpr (RowState<T, L, VEC, WM>::kPacked) {
    // z = 1{x > 0} = 1 - 1{x <= 0} unlifted; z = 1{x >= 0} = 1{-x <= 0} lifted
    const uint32_t flip = lifted ? 0x80008000u : 0u, inv = lifted ? 0u : 0x00010001u;
    uint32_t wd[VEC / 2];
    raw_words(xr[0], wd);
    uint32_t zm = 0;
#pragma unroll
    for (int k = 0; k < VEC / 2; ++k) {
      const uint32_t z = __builtin_bit_cast(uint32_t, nonpos_pair(wd[k] ^ flip)) ^ inv;
      zm |= ((z & 1u) | ((z >> 15) & 2u)) << (2 * k);
    }
    st.zm = zm;
  } else {
    st.zm = side_mask_raw<T, VEC, L>(xr, lifted);
  }
  reset_counters(st);
}

// Takes one neighbour slot: w * x_u into the sums and, when scoring, w and w z_u into the
// counters. Unlifted bfloat16 rows with unit or +-1 weights stay packed: the sums use the
// bfloat16 dot instruction against (w, 0) / (0, w), and the counters add w 1{x_u <= 0}
// per 16-bit lane (z_u = 1{x_u > 0} is its complement). Lifted rows with l = 1 have
// z_u = 1{x_u >= 0} = 1{-x_u <= 0}: the same count taken on -x_u (sign bits flipped).
template <typename T, int VEC, int L, int WM>
__device__ __forceinline__ void take_slot(RowState<T, L, VEC, WM>& st, const typename VecIO<T, VEC>::raw (&xr)[L],
                                          float wq, bool do_score, int lifted) {
  using ST = typename ScoreType<WM>::type;
  if constexpr (RowState<T, L, VEC, WM>::kPacked) {
    uint32_t wd[VEC / 2];
    raw_words(xr[0], wd);
    const uint32_t wlo = WM == kUnitW ? st.ulo : (__float_as_uint(wq) >> 16);
    const uint32_t whi = WM == kUnitW ? st.uhi : wlo << 16;
#pragma unroll
    for (int k = 0; k < VEC / 2; ++k) {
      st.acc[0][2 * k] = dot2_bf16(wd[k], wlo, st.acc[0][2 * k]);
      st.acc[0][2 * k + 1] = dot2_bf16(wd[k], whi, st.acc[0][2 * k + 1]);
    }
    if (do_score) {
      const uint32_t flip = lifted ? 0x80008000u : 0u;
      const short ws = (short)(WM == kUnitW ? 1 : (wq < 0.0f ? -1 : 1));
#pragma unroll
      for (int k = 0; k < VEC / 2; ++k) {
        const i16x2 z = nonpos_pair(wd[k] ^ flip);
        if (WM == kUnitW)
          st.zp[k] += z;
        else
          st.zp[k] += z * i16x2{ws, ws};
      }
    }
  } else if constexpr (sizeof(T) == 2 && VEC >= 2 && (WM == kUnitW || WM == kPm1W)) {
    // bfloat16 rows of l > 1 components with unit or +-1 weights: the sums with the dot
    // instruction from the raw words; values are unpacked only to score
    const uint32_t wlo = WM == kUnitW ? st.ulo : (__float_as_uint(wq) >> 16);
    const uint32_t whi = WM == kUnitW ? st.uhi : wlo << 16;
#pragma unroll
    for (int i = 0; i < L; ++i) {
      uint32_t wd[VEC / 2];
      raw_words(xr[i], wd);
#pragma unroll
      for (int k = 0; k < VEC / 2; ++k) {
        st.acc[i][2 * k] = dot2_bf16(wd[k], wlo, st.acc[i][2 * k]);
        st.acc[i][2 * k + 1] = dot2_bf16(wd[k], whi, st.acc[i][2 * k + 1]);
      }
    }
    if (do_score) {
      float xu[L][VEC];
#pragma unroll
      for (int i = 0; i < L; ++i) VecIO<T, VEC>::unpack(xr[i], xu[i]);
      const uint32_t sm = side_mask<L, VEC>(xu, lifted);
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int bit = (int)((sm >> e) & 1u);
        st.zs[e] += WM == kUnitW ? bit : (wq < 0.0f ? -bit : bit);
      }
    }
  } else {
    float xu[L][VEC];
#pragma unroll
    for (int i = 0; i < L; ++i) VecIO<T, VEC>::unpack(xr[i], xu[i]);
#pragma unroll
    for (int i = 0; i < L; ++i)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        if (WM == kUnitW)
          st.acc[i][e] += xu[i][e];
        else
          st.acc[i][e] = fmaf(wq, xu[i][e], st.acc[i][e]);
      }
    if (do_score) {
      const uint32_t sm = side_mask<L, VEC>(xu, lifted);
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const uint32_t bit = (sm >> e) & 1u;
        if (WM == kUnitW)
          st.zs[e] += (int)bit;
        else if (WM == kRealW)
          st.zs[e] += bit ? wq : 0.0f;
        else
          st.zs[e] += (int)bit * (int)wq;
      }
    }
  }
  if constexpr (WM != kUnitW) st.wsum += (ST)wq;
}

// One window of the team's slot range: slots [p, min(p + W, pe)) of the staged list. All
// gathers of the window are issued before any is used; then the slots are folded in list
// order: a self slot (SELF lists only) closes the open row and opens its own, a neighbour
// slot is taken into the open row.
// Element offset of a gathered node's row (the slot's flag bit is ignored). Lanes of
// several elements run only where n < 2^24 and n * C < 2^32 (the host keeps larger graphs
// on one-element lanes): one full-rate 24-bit multiply instead of a 64-bit one.
template <int VEC>
__device__ __forceinline__ size_t row_offset(int slot, int C) {
  if constexpr (VEC == 1) return (size_t)((uint32_t)slot & 0x7FFFFFFFu) * (size_t)C;
  else return (size_t)(uint32_t)__umul24((uint32_t)slot, (uint32_t)C);
}

// Gathered values of component i of a neighbour row. Lifted rows skip the components at
// and past the active count na: those are exactly 0 in every row (the start writes zeros
// and a zero neighbour sum keeps them there), so the skipped load is replaced by its known
// value and the step's results are unchanged bit for bit. ALL: every component is active
// (no predicate on the loads).
template <typename T, int VEC, int L, bool ALL>
__device__ __forceinline__ typename VecIO<T, VEC>::raw gather_comp(const T* p, int i, int na) {
  if constexpr (ALL || L == 1) {
    return VecIO<T, VEC>::load_raw(p);
  } else {
    typename VecIO<T, VEC>::raw v{};
    if (i < na) v = VecIO<T, VEC>::load_raw(p);
    return v;
  }
}

template <typename T, int VEC, int L, int WM, bool SELF, bool ALL>
__device__ __forceinline__ void gather_window(const StepArgs& a, const T* __restrict__ X, T* __restrict__ Y,
                                              uint8_t* __restrict__ bw, const int* s_slot, const float* s_sw,
                                              float* s_part, int part_idx, int p, int pe, int bl, int lc, int gb,
                                              const float* __restrict__ eta, RowState<T, L, VEC, WM>& st,
                                              ScoreAcc<T, L, VEC, WM>& sc, bool do_score, int lifted, float* vel,
                                              int na) {
  using IO = VecIO<T, VEC>;
  constexpr int W = Tune<T, L, VEC>::W;
  const size_t B = (size_t)a.B;
  static_assert(W <= kSlotPad, "window reads past the staged slots");
  // branch-free slot reads: past the share they are the next team's slots or, past the
  // item's last slot, the zero padding (row 0); those gathers are in bounds and not folded
  const int rem = pe - p;
  int sl[W];
#pragma unroll
  for (int q = 0; q < W; ++q) sl[q] = s_slot[p + q];
  typename IO::raw xr[W][L];
#pragma unroll
  for (int q = 0; q < W; ++q) {
    // slots past the share are gathered (in bounds) and not folded: no branch per load
#pragma unroll
    for (int i = 0; i < L; ++i) xr[q][i] = gather_comp<T, VEC, L, ALL>(X + row_offset<VEC>(sl[q], a.C) + i * B + bl, i, na);
  }
  if (st.lazy) {
    st.zm = side_mask_raw<T, VEC, L>(st.xv, lifted);
    st.lazy = false;
  }
#pragma unroll
  for (int q = 0; q < W; ++q) {
    if (q < rem) {
      const float wq = WM == kUnitW ? 1.0f : s_sw[p + q];
      if (SELF && sl[q] < 0) {
        if (st.row >= 0)
          close_row<T, VEC, L, WM>(a, Y, bw, s_part, part_idx, do_score, bl, lc, gb, eta, st, sc, p + q, lifted, vel);
        open_row<T, L, VEC, WM>(st, sl[q] & 0x7FFFFFFF, xr[q], wq, lifted, p + q);
      } else {
        take_slot<T, VEC, L, WM>(st, xr[q], wq, do_score, lifted);
      }
    }
  }
}

// Software-pipelined windows of the normal path of lifted rows: the gathers of the next
// window are in flight while the current one is folded. Two buffers of PW slots with fixed names (the
// loop is unrolled by two, so both stay in registers), at most 128 bytes of gathered
// values per lane each.
template <typename T, int L, int VEC>
struct PipeTune {
  static constexpr int kRawBytes = (int)sizeof(typename VecIO<T, VEC>::raw) * L;
  static constexpr int W0 = Tune<T, L, VEC>::W;
  static constexpr int W1 = VEC == 1 ? W0 / 2 : W0;  // one-element lanes: the slot indices count too
  static constexpr int W = W1 * kRawBytes <= 128 ? W1 : (128 / kRawBytes < 1 ? 1 : 128 / kRawBytes);
};

template <typename T, int VEC, int L, int PW>
struct WinBuf {
  int sl[PW];
  typename VecIO<T, VEC>::raw xr[PW][L];
};

template <typename T, int VEC, int L, int PW, bool ALL>
__device__ __forceinline__ void load_window(const StepArgs& a, const T* __restrict__ X, const int* s_slot, int p,
                                            int pe, int bl, int na, WinBuf<T, VEC, L, PW>& wb) {
  using IO = VecIO<T, VEC>;
  const size_t B = (size_t)a.B;
  (void)pe;
#pragma unroll
  for (int q = 0; q < PW; ++q) wb.sl[q] = s_slot[p + q];
#pragma unroll
  for (int q = 0; q < PW; ++q) {
    // slots past the share are gathered (in bounds) and not folded: no branch per load
#pragma unroll
    for (int i = 0; i < L; ++i) wb.xr[q][i] = gather_comp<T, VEC, L, ALL>(X + row_offset<VEC>(wb.sl[q], a.C) + i * B + bl, i, na);
  }
}

template <typename T, int VEC, int L, int WM, int PW>
__device__ __forceinline__ void fold_window(const StepArgs& a, T* __restrict__ Y, uint8_t* __restrict__ bw,
                                            const float* s_sw, float* s_part, int part_idx, int p, int pe, int bl,
                                            int lc, int gb, const float* __restrict__ eta,
                                            const WinBuf<T, VEC, L, PW>& wb, RowState<T, L, VEC, WM>& st,
                                            ScoreAcc<T, L, VEC, WM>& sc, bool do_score, int lifted, float* vel) {
  if (st.lazy) {
    st.zm = side_mask_raw<T, VEC, L>(st.xv, lifted);
    st.lazy = false;
  }
  const int rem = pe - p;
#pragma unroll
  for (int q = 0; q < PW; ++q) {
    if (q < rem) {
      const float wq = WM == kUnitW ? 1.0f : s_sw[p + q];
      if (wb.sl[q] < 0) {
        if (st.row >= 0)
          close_row<T, VEC, L, WM>(a, Y, bw, s_part, part_idx, do_score, bl, lc, gb, eta, st, sc, p + q, lifted, vel);
        open_row<T, L, VEC, WM>(st, wb.sl[q] & 0x7FFFFFFF, wb.xr[q], wq, lifted, p + q);
      } else {
        take_slot<T, VEC, L, WM>(st, wb.xr[q], wq, do_score, lifted);
      }
    }
  }
}

// Completion of scored step s for the (graph, initialisation) pairs of the 256-wide blocks
// blk, blk + nblk, ...: the R replicas of acc[s & 1] are summed in replica order and
// cleared, cut = a.cut_scale * sum goes to cur_cut and the trace, a strictly larger cut
// replaces the best cut (best step s), and the improvements go to mask[s & 1]. Every
// thread of the workgroup calls it (blockDim.x = 256).
constexpr int kMaxReplicas = 16;
__device__ __forceinline__ void finish_scores(const StepArgs& a, long long s, int blk, int nblk) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int GB = a.G * a.B;
  double* acc = a.acc + (size_t)(s & 1) * a.R * GB;
  uint8_t* mask = a.mask + (size_t)(s & 1) * a.G * a.NBY;
  const int chunk = a.B < 8 ? a.B : 8;
  for (int base = blk * 256; base < GB; base += nblk * 256) {
    const int idx = base + tid;
    const bool in = idx < GB;
    bool imp = false;
    if (in) {
      // all replica loads in flight together, summed in replica order
      double v[kMaxReplicas];
#pragma unroll
      for (int r = 0; r < kMaxReplicas; ++r)
        v[r] = r < a.R ? __hip_atomic_load(acc + (size_t)r * GB + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                       : 0.0;
      double sum = 0.0;
#pragma unroll
      for (int r = 0; r < kMaxReplicas; ++r) sum += v[r];
#pragma unroll
      for (int r = 0; r < kMaxReplicas; ++r)
        if (r < a.R) __hip_atomic_store(acc + (size_t)r * GB + idx, 0.0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const double cut = a.cut_scale * sum;
      a.cur_cut[idx] = cut;
      if (a.trace) a.trace[(size_t)(s % a.trace_cap) * GB + idx] = cut;
      imp = cut > a.best_cut[idx];
      if (imp) {
        a.best_cut[idx] = cut;
        a.best_step[idx] = (int)s;
      }
    }
    const unsigned long long bal = __ballot(imp);
    if (in && (idx % chunk) == 0) {
      const int g = idx / a.B, b = idx % a.B;
      mask[g * a.NBY + (b >> 3)] = (uint8_t)((bal >> lane) & ((1ull << chunk) - 1ull));
    }
  }
}

// End of one step launch: two-level ticket (per XCD, then global), and the last workgroup
// advances the control block. Inside a launch, workgroups exchange data only through
// device-scope atomics (score accumulators, tickets); plain stores (iterate, bits, cuts)
// are consumed by later launches, after the kernel boundary. Immediate mode (nextra = 0):
// every lane first waits until its own score atomics are acknowledged and the last
// workgroup completes step t itself. Lagged mode: step t is completed by the extra
// workgroups of the next launch, so nothing waits here. cp is the step whose completion
// this launch's extra workgroups ran (read from the control block at the start). Every
// workgroup of the grid must call this exactly once.
__device__ __forceinline__ void complete_step(const StepArgs& a, long long t, bool do_score, long long cp,
                                              int& s_last) {
  const int tid = threadIdx.x;
  const int xcd = blockIdx.x & 7;
  const int nbx = ((int)gridDim.x - xcd + 7) >> 3;
  const bool lag = a.nextra > 0;
  if (!lag) __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0) {
    bool last = false;
    const unsigned p = atomicAdd(&a.ctrl->xticket[xcd][0], 1u);
    if (p == (unsigned)nbx - 1u) {
      const unsigned nx = gridDim.x < 8u ? gridDim.x : 8u;  // XCDs that received workgroups
      const unsigned q = atomicAdd(&a.ctrl->ticket, 1u);
      last = (q == nx - 1u);
    }
    s_last = last;
  }
  __syncthreads();
  if (!s_last) return;
  if (!lag && do_score) finish_scores(a, t, 0, 1);
  if (tid < 8) a.ctrl->xticket[tid][0] = 0u;
  if (tid == 0) {
    if (lag) {
      a.ctrl->fpend = cp;
      a.ctrl->cpend = do_score ? t : -1;
    } else {
      a.ctrl->fpend = do_score ? t : -1;
      a.ctrl->cpend = -1;
    }
    if (a.do_update) a.ctrl->t = t + 1;
    a.ctrl->ticket = 0u;
  }
}

#ifndef DECO_STEP_WAVES_PER_EU
#define DECO_STEP_WAVES_PER_EU 3
#endif

// LF: the lifted flag known when compiling (0 or 1, rows of one component) or -1 (read from a).
// MOM: heavy-ball momentum (velocity in a.vel); without it the update code has no velocity path.
// ALL: l > 1 rows gather every component without predicates (4-value lanes of up to 4
// components: the launch runs the largest active count, and the components of an
// initialisation with fewer are gathered as the zeros they are).
template <typename T, int VEC, int L, int WM, int LF, bool MOM, bool ALL = false>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(DECO_STEP_WAVES_PER_EU)))
void k_step(StepArgs a) {
  constexpr int W = Tune<T, L, VEC>::W;
  using ST = typename ScoreType<WM>::type;
  using IO = VecIO<T, VEC>;
  __shared__ int s_slot[kEmax + kSlotPad];
  __shared__ float s_sw[WM == kUnitW ? 1 : kEmax];
  __shared__ int s_rp[kRmax + 1];
  __shared__ __align__(16) float s_eta[512];
  // score flush (double per initialisation of the tile per wave) / partial sums of the
  // teams (float per lane, component and initialisation) / long-row reduction (float per
  // component and initialisation of the tile per wave)
  constexpr int kRedBytes = kWaves * (L * 256 * 4 > 256 * 8 ? L * 256 * 4 : 256 * 8);
  static_assert(kThreads * L * VEC * 4 <= kRedBytes, "partial sums of the teams");
  __shared__ __align__(16) unsigned char s_red_raw[kRedBytes];
  __shared__ int s_last;
  double* s_red = reinterpret_cast<double*>(s_red_raw);
  float* s_acc = reinterpret_cast<float*>(s_red_raw);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int Wc = a.Wc;
  // Wc, the team count NS and the replica count R are powers of two: shifts and masks
  const int wl = __builtin_ctz((unsigned)Wc);
  const int nsl = 8 - wl;        // log2 of the team count (kThreads = 256)
  const int NS = kThreads >> wl; // row teams (sub-groups of Wc lanes) per workgroup
  const int lc = tid & (Wc - 1);
  const int sgi = tid >> wl;

  const int lifted = LF >= 0 ? LF : a.lifted;
  float* const vel = MOM ? a.vel : nullptr;
  const long long t = a.ctrl->t;
  const bool do_score = a.force_score || (t % a.ctrl->score_every) == 0;
  const long long cp = a.ctrl->cpend;  // step completed by the extra workgroups of this launch
  const long long fp = a.ctrl->fpend;  // step whose improvements this launch folds
  // the extra workgroups after the work grid complete step cp, off the critical path
  const int gw = (int)gridDim.x - a.nextra;
  if ((int)blockIdx.x >= gw) {
    if (cp >= 0) finish_scores(a, cp, (int)blockIdx.x - gw, a.nextra);
    complete_step(a, t, do_score, cp, s_last);
    return;
  }
  const int par = (int)(t & 1);
  const T* __restrict__ X = reinterpret_cast<const T*>(a.x[par]);
  T* __restrict__ Y = reinterpret_cast<T*>(a.x[par ^ 1]);
  uint8_t* __restrict__ bw = a.bits[t % 3];
  const uint8_t* bm = fp >= 0 ? a.bits[fp % 3] : nullptr;
  const uint8_t* fmask = a.mask + (size_t)(fp & 1) * a.G * a.NBY;
  double* acc = a.acc + (size_t)(t & 1) * a.R * a.G * a.B;
  const int Bt = Wc * VEC;
  const int gb = VEC >= 8 ? 1 : (8 / VEC < Wc ? 8 / VEC : Wc);

  const int xcd = blockIdx.x & 7;
  const int kb = blockIdx.x >> 3;
  const int nbx = (gw - xcd + 7) >> 3;
  const int it0 = a.seg[xcd], it1 = a.seg[xcd + 1];

  ScoreAcc<T, L, VEC, WM> sc;
  sc.clear();
  int cg = -1, cbt = -1;

  // score partials of the current (graph, tile): wave, then workgroup, then one atomic per
  // initialisation into replica blockIdx % R. Every thread of the workgroup calls it.
  auto flush = [&]() {
    double d[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      d[e] = sc.get(e);
      for (int s = Wc; s < 64; s <<= 1) d[e] += __shfl_xor(d[e], s);
    }
    __syncthreads();
    if (lane < Wc) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) s_red[wv * 256 + lane * VEC + e] = d[e];
    }
    __syncthreads();
    for (int j = tid; j < Bt; j += kThreads) {
      double v = s_red[j];
#pragma unroll
      for (int q = 1; q < kWaves; ++q) v += s_red[q * 256 + j];
      if (v != 0.0) {
        double* dst = acc + ((size_t)(blockIdx.x & (a.R - 1)) * a.G + cg) * a.B + (size_t)cbt * Bt + j;
        unsafeAtomicAdd(dst, v);
      }
    }
    sc.clear();
  };

  for (int it = it0 + kb;; it += nbx) {
    const bool have = it < it1;
    int4 hd = make_int4(0, 0, 0, 0), tl = make_int4(0, 0, 0, 0);
    if (have) {
      hd = a.items[2 * it];
      tl = a.items[2 * it + 1];
    }
    if (do_score && cg >= 0) flush();
    if (!have) break;
    const int x = hd.x, y = hd.y, s0 = hd.z, s1 = hd.w;
    const bool longrow = tl.z != 0;
    cg = tl.x;
    cbt = tl.y;
    const int bl = cbt * Bt + lc * VEC;  // first initialisation of this lane
    // lifted rows: components gathered per neighbour (the largest active count among the
    // lane's initialisations; the rest are exactly 0)
    int na = L;
    if constexpr (L > 1 && !ALL) {
      if (a.lact) {
        na = 0;
#pragma unroll
        for (int e = 0; e < VEC; ++e) na = max(na, bl + e < a.B ? a.lact[bl + e] : 0);
        // the wave's largest count, held in a scalar register (gathering a component that
        // is 0 everywhere changes nothing): the load predicates are uniform branches
        for (int o = 32; o > 0; o >>= 1) na = max(na, __shfl_xor(na, o));
        na = __builtin_amdgcn_readfirstlane(na);
      }
    }
    // the improvement mask word this thread folds at the end of the item (word-aligned rows
    // and tiles: a thread's words all lie in one tile column, since TW divides kThreads)
    const int fTB = Bt >= 8 ? (Bt >> 3) : 1, fb0 = (cbt * Bt) >> 3;
    const bool fwords = (a.NBY & 3) == 0 && (fTB & 3) == 0;
    const int fTW = fTB >> 2;
    uint32_t fold_m = 0u;
    if (fp >= 0 && fwords)
      fold_m = reinterpret_cast<const uint32_t*>(fmask)[(size_t)cg * (a.NBY >> 2) + (fb0 >> 2) + (tid & (fTW - 1))];
    __syncthreads();  // LDS of the previous item is free
    // step sizes of the tile (read by the row updates after the staging barrier)
    for (int j = tid; j < Bt; j += kThreads) {
      const float et = a.eta[cbt * Bt + j];
      s_eta[j] = et;
      s_eta[256 + j] = et * a.cW;
    }
    const float* eta = s_eta + lc * VEC;

    if (!longrow) {
      const int E = s1 - s0, R = y - x;
      for (int k = tid; k < E; k += kThreads) {
        s_slot[k] = a.slots[s0 + k];
        if (WM != kUnitW) s_sw[k] = a.sw[s0 + k];
      }
      if (tid < kSlotPad) s_slot[E + tid] = 0;  // windows past the last slot gather row 0
      for (int i = tid; i <= R; i += kThreads) s_rp[i] = a.rp[x + i] + x + i - s0;
      __syncthreads();
      // merge-path split: the team takes exactly the slots [c0, c1); a row cut by a share
      // boundary is finished by the team holding its own slot, which adds the partial sums
      // of the following teams in team order after a barrier
      const int c0 = (E * sgi) >> nsl;
      const int c1 = (E * (sgi + 1)) >> nsl;
      const int part_idx = (sgi * Wc + lc) * (L * VEC);
      RowState<T, L, VEC, WM> st;
      st.set_unit_pairs();
      st.row = -1;
      st.zm = 0u;
      st.dsum = 0.0f;
      st.head = false;
      st.lazy = false;
      st.open = c0;
      reset_counters(st);
      if (c0 < c1) {
        int lo = 0, hi = R;  // first row starting after c0
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (s_rp[mid] <= c0) lo = mid + 1; else hi = mid;
        }
        if (s_rp[lo - 1] < c0) {
          // the share starts inside row x + lo - 1: its values give the sides for scoring
          st.row = x + lo - 1;
          st.head = true;
          st.lazy = true;
          st.open = c0;
#pragma unroll
          for (int i = 0; i < L; ++i) {
            st.xv[i] = IO::load_raw(X + (size_t)st.row * a.C + (size_t)i * a.B + bl);
#pragma unroll
            for (int e = 0; e < VEC; ++e) st.acc[i][e] = 0.0f;
          }
        }
      }
      if constexpr (L == 1) {
        // unlifted rows: one window at a time (their folds are short; the loads of a window
        // are waited for one by one)
        for (int p = c0; p < c1; p += W)
          gather_window<T, VEC, L, WM, true, true>(a, X, Y, bw, s_slot, s_sw, s_acc, part_idx, p, c1, bl, lc, gb, eta,
                                                   st, sc, do_score, lifted, vel, na);
      } else {
        // lifted rows: the next window's gathers are in flight during each fold
        constexpr int PW = PipeTune<T, L, VEC>::W;
        static_assert(3 * PW <= kSlotPad, "windows read past the staged slots");
        WinBuf<T, VEC, L, PW> wa, wb;
        load_window<T, VEC, L, PW, ALL>(a, X, s_slot, c0, c1, bl, na, wa);
        for (int p = c0; p < c1; p += 2 * PW) {
          load_window<T, VEC, L, PW, ALL>(a, X, s_slot, p + PW, c1, bl, na, wb);
          fold_window<T, VEC, L, WM, PW>(a, Y, bw, s_sw, s_acc, part_idx, p, c1, bl, lc, gb, eta, wa, st, sc,
                                         do_score, lifted, vel);
          load_window<T, VEC, L, PW, ALL>(a, X, s_slot, p + 2 * PW, c1, bl, na, wa);
          fold_window<T, VEC, L, WM, PW>(a, Y, bw, s_sw, s_acc, part_idx, p + PW, c1, bl, lc, gb, eta, wb, st, sc,
                                         do_score, lifted, vel);
        }
      }
      bool tail = false;
      int next = 0;
      if (st.row >= 0) {
        if (st.head) {
          close_row<T, VEC, L, WM>(a, Y, bw, s_acc, part_idx, do_score, bl, lc, gb, eta, st, sc, c1, lifted, vel);
        } else {
          const int i = st.row - x;
          next = s_rp[i + 1];
          if (next <= c1) {
            close_row<T, VEC, L, WM>(a, Y, bw, s_acc, part_idx, do_score, bl, lc, gb, eta, st, sc, c1, lifted, vel);
          } else {
            // the row continues in later shares: score this share now, update after them
            tail = true;
            if constexpr (WM == kUnitW) st.wsum = c1 - st.open;
            if (do_score) close_score(st, sc, lifted);
            if (WM == kUnitW) st.dsum = (float)(next - s_rp[i] - 1);
          }
        }
      }
      __syncthreads();
      if (tail) {
        for (int k = sgi + 1; k < NS; ++k) {
          const int k0 = (E * k) >> nsl, k1 = (E * (k + 1)) >> nsl;
          if (k0 >= next) break;
          if (k0 < k1) {
            const int idx = (k * Wc + lc) * (L * VEC);
#pragma unroll
            for (int i = 0; i < L; ++i)
#pragma unroll
              for (int e = 0; e < VEC; ++e) st.acc[i][e] += s_acc[idx + i * VEC + e];
          }
        }
        finish_row<T, VEC, L, WM>(a, Y, bw, do_score, true, bl, lc, gb, eta, st, vel);
      }
    } else {
      // one long row: every team takes a contiguous share of each staged chunk of its
      // neighbour slots; the partial sums are reduced in a fixed order
      RowState<T, L, VEC, WM> st;
      st.set_unit_pairs();
      st.row = x;
#pragma unroll
      for (int i = 0; i < L; ++i) {
        st.xv[i] = IO::load_raw(X + (size_t)x * a.C + (size_t)i * a.B + bl);
#pragma unroll
        for (int e = 0; e < VEC; ++e) st.acc[i][e] = 0.0f;
      }
      st.dsum = WM == kUnitW ? (float)(s1 - s0 - 1) : a.sw[s0];
      st.zm = 0u;
      st.head = false;
      st.lazy = false;
      reset_counters(st);
      for (int sb = s0 + 1; sb < s1; sb += kEmax) {
        const int E = (s1 - sb) < kEmax ? (s1 - sb) : kEmax;
        if (sb != s0 + 1) __syncthreads();
        for (int k = tid; k < E; k += kThreads) {
          s_slot[k] = a.slots[sb + k];
          if (WM != kUnitW) s_sw[k] = a.sw[sb + k];
        }
        if (tid < kSlotPad) s_slot[E + tid] = 0;
        __syncthreads();
        st.zm = side_mask_raw<T, VEC, L>(st.xv, lifted);
        const int c0 = (E * sgi) >> nsl;
        const int c1 = (E * (sgi + 1)) >> nsl;
        for (int p = c0; p < c1; p += W)
          gather_window<T, VEC, L, WM, false, ALL>(a, X, Y, bw, s_slot, s_sw, s_acc, 0, p, c1, bl, lc, gb, eta, st,
                                                   sc, do_score, lifted, vel, na);
        // score of this chunk's share; the 16-bit partials hold at most one chunk
        if (do_score) {
          if constexpr (WM == kUnitW) st.wsum = c1 - c0;
          close_score(st, sc, lifted);
          flush();
        }
      }
      st.zm = side_mask_raw<T, VEC, L>(st.xv, lifted);
      // teams of one wave first (butterfly), then the waves in order through LDS
#pragma unroll
      for (int i = 0; i < L; ++i)
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          for (int s = Wc; s < 64; s <<= 1) st.acc[i][e] += __shfl_xor(st.acc[i][e], s);
      __syncthreads();
      if (lane < Wc) {
#pragma unroll
        for (int i = 0; i < L; ++i)
#pragma unroll
          for (int e = 0; e < VEC; ++e) s_acc[wv * (L * 256) + (lane * L + i) * VEC + e] = st.acc[i][e];
      }
      __syncthreads();
      if (wv == 0) {
#pragma unroll
        for (int q = 1; q < kWaves; ++q)
#pragma unroll
          for (int i = 0; i < L; ++i)
#pragma unroll
            for (int e = 0; e < VEC; ++e) st.acc[i][e] += s_acc[q * (L * 256) + (lc * L + i) * VEC + e];
      }
      finish_row<T, VEC, L, WM>(a, Y, bw, do_score, sgi == 0, bl, lc, gb, eta, st, vel);
    }

    // fold the previous scored step's improvements into best_bits for this item's rows and
    // tile (the bit slot bm is rewritten only by the launch after this one): 4-byte words
    // when rows and tiles are word aligned, all loads of a batch in flight together
    if (fp >= 0) {
      const int TB = fTB;
      const int b0 = fb0;
      const int R = y - x;
      if (fwords) {
        constexpr int kU = 8;
        const int TW = fTW, NW = a.NBY >> 2, twl = __builtin_ctz((unsigned)TW);  // TW: a power of two
        const uint32_t* bm32 = reinterpret_cast<const uint32_t*>(bm);
        uint32_t* best32 = reinterpret_cast<uint32_t*>(a.best_bits);
        for (int base = 0; fold_m != 0u && base < R * TW; base += kThreads * kU) {
          uint32_t mo[kU], mb[kU];
          size_t wi[kU];
          bool in[kU];
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const int k = base + u * kThreads + tid;
            const int r = k >> twl, c = k & (TW - 1);
            in[u] = k < R * TW;
            wi[u] = (size_t)(x + r) * NW + (b0 >> 2) + c;
          }
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            mo[u] = in[u] ? bm32[wi[u]] : 0u;
            mb[u] = in[u] ? best32[wi[u]] : 0u;
          }
#pragma unroll
          for (int u = 0; u < kU; ++u)
            if (in[u]) best32[wi[u]] = (mb[u] & ~fold_m) | (mo[u] & fold_m);
        }
      } else {
        for (int k = tid; k < R * TB; k += kThreads) {
          const int r = k / TB, bb = b0 + k % TB;
          const uint32_t m = fmask[cg * a.NBY + bb];
          if (m) {
            const size_t bi = (size_t)(x + r) * a.NBY + bb;
            a.best_bits[bi] = (uint8_t)((a.best_bits[bi] & ~m) | (bm[bi] & m));
          }
        }
      }
    }
  }

  complete_step(a, t, do_score, cp, s_last);
}


// ------------------------------------------------------------------ dense graphs: MFMA path
// For a dense graph the gradient W X is a true GEMM. One launch computes, for a 128-row by
// 128-column tile of X,
//   P = W X  and  Q = W S,  S = sign(X) in {-1, +1}   (bfloat16 operands, float32 accumulation)
// with v_mfma_f32_32x32x16_bf16 (4 waves, each 64 x 64 of P and of Q as 2 x 2 MFMA blocks).
// Both operands stream with k contiguous: W's rows, and the rows of a transposed copy XT of X
// (C x n) that every step writes next to X; K steps of 64 are double-buffered through LDS and
// the sign fragments are formed in registers from the X fragments. Workgroups of one XCD take
// consecutive tiles, so the tiles sharing a W row panel meet in that XCD's L2. P finishes the
// projected update; Q scores exactly: with s = 2z - 1,
//   sum_u w_vu 1{z_u != z_v} = (d_w(v) - s_v (W s)_v) / 2,
// and W s is exact in float32 for integer weights whose row sums of |w| stay within 2^24
// (checked when the handle is made), so each tile
// adds sum_v (d_w(v) - s_v (W s)_v) per column (in double) and the cut is 1/4 of the total. The epilogue
// stages the tile in LDS and writes X_t+1 and its transpose with 16-byte stores, the cut bits
// and the fold of the previous step's improvements into best_bits.
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16_t;

constexpr int kDBM = 128, kDBN = 128, kDBK = 64, kDLd = kDBK + 8;  // LDS row: 144 bytes
constexpr int kDEp = kDBN + 8;                                      // epilogue row: 272 bytes

// Signs (+1 / -1 as bfloat16, x > 0 ? +1 : -1) of the 8 bfloat16 of an MFMA fragment.
__device__ __forceinline__ bf16x8_t sign_frag(const bf16x8_t& f) {
  const uint4 w = __builtin_bit_cast(uint4, f);
  uint4 s;
  s.x = 0x3F803F80u | (__builtin_bit_cast(uint32_t, nonpos_pair(w.x)) << 15);
  s.y = 0x3F803F80u | (__builtin_bit_cast(uint32_t, nonpos_pair(w.y)) << 15);
  s.z = 0x3F803F80u | (__builtin_bit_cast(uint32_t, nonpos_pair(w.z)) << 15);
  s.w = 0x3F803F80u | (__builtin_bit_cast(uint32_t, nonpos_pair(w.w)) << 15);
  return __builtin_bit_cast(bf16x8_t, s);
}

struct DStage {
  uint4 a0, a1, a2, a3, b0, b1, b2, b3;
};

// One K step of W rows and XT rows (64 bytes per thread each), as values.
__device__ __forceinline__ DStage dense_gload2(const uint16_t* __restrict__ W, const uint16_t* __restrict__ XT, int n,
                                               int row0, int col0, int k0, int tid) {
  const uint4* pa = reinterpret_cast<const uint4*>(W + (size_t)(row0 + (tid >> 1)) * n + k0 + (tid & 1) * 32);
  const uint4* pb = reinterpret_cast<const uint4*>(XT + (size_t)(col0 + (tid >> 1)) * n + k0 + (tid & 1) * 32);
  DStage d;
  d.a0 = pa[0];
  d.a1 = pa[1];
  d.a2 = pa[2];
  d.a3 = pa[3];
  d.b0 = pb[0];
  d.b1 = pb[1];
  d.b2 = pb[2];
  d.b3 = pb[3];
  return d;
}

__device__ __forceinline__ void dense_sstore2(uint16_t (*As)[kDLd], uint16_t (*Bs)[kDLd], int tid, const DStage& d) {
  uint4* da = reinterpret_cast<uint4*>(&As[tid >> 1][(tid & 1) * 32]);
  uint4* db = reinterpret_cast<uint4*>(&Bs[tid >> 1][(tid & 1) * 32]);
  da[0] = d.a0;
  da[1] = d.a1;
  da[2] = d.a2;
  da[3] = d.a3;
  db[0] = d.b0;
  db[1] = d.b1;
  db[2] = d.b2;
  db[3] = d.b3;
}

// The 4 k16 sub-steps of one staged K step: P += A B, Q += A sign(B) for this wave's 64 x 64.
__device__ __forceinline__ void dense_mma_stage(const uint16_t (*As)[kDLd], const uint16_t (*Bs)[kDLd], int wm, int wn,
                                                int lo, int hi, f32x16_t (&P)[2][2], f32x16_t (&Q)[2][2]) {
#pragma unroll
  for (int ks = 0; ks < kDBK / 16; ++ks) {
    bf16x8_t fa[2], fb[2], fs[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      fa[i] = *reinterpret_cast<const bf16x8_t*>(&As[wm * 64 + i * 32 + lo][ks * 16 + 8 * hi]);
      fb[i] = *reinterpret_cast<const bf16x8_t*>(&Bs[wn * 64 + i * 32 + lo][ks * 16 + 8 * hi]);
      fs[i] = sign_frag(fb[i]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        P[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fb[j], P[i][j], 0, 0, 0);
        Q[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i], fs[j], Q[i][j], 0, 0, 0);
      }
  }
}

__global__ __launch_bounds__(256) void k_dense_step(StepArgs a) {
  __shared__ __align__(16) uint16_t smem[2 * 2 * kDBM * kDLd];  // A and B stages; the epilogue's tiles
  __shared__ float s_dw[kDBM];
  __shared__ double s_col[2][kDBN];
  __shared__ int s_last;
  uint16_t (*As)[kDBM][kDLd] = reinterpret_cast<uint16_t (*)[kDBM][kDLd]>(smem);
  uint16_t (*Bs)[kDBM][kDLd] = reinterpret_cast<uint16_t (*)[kDBM][kDLd]>(smem + 2 * kDBM * kDLd);
  uint16_t (*Xs)[kDEp] = reinterpret_cast<uint16_t (*)[kDEp]>(smem);              // X_t tile
  uint16_t (*Ys)[kDEp] = reinterpret_cast<uint16_t (*)[kDEp]>(smem + kDBM * kDEp);  // X_t+1 tile

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1, hi = lane >> 5, lo = lane & 31;
  const long long t = a.ctrl->t;
  const bool do_score = a.force_score || (t % a.ctrl->score_every) == 0;
  const long long cp = a.ctrl->cpend;
  const long long fp = a.ctrl->fpend;  // step whose improvements this launch folds
  const uint8_t* fbits = fp >= 0 ? a.bits[fp % 3] : nullptr;
  const uint8_t* fmask = a.mask + (size_t)(fp & 1) * a.NBY;
  const int par = (int)(t & 1);
  const uint16_t* __restrict__ X = reinterpret_cast<const uint16_t*>(a.x[par]);
  uint16_t* __restrict__ Y = reinterpret_cast<uint16_t*>(a.x[par ^ 1]);
  const uint16_t* __restrict__ XT = reinterpret_cast<const uint16_t*>(a.xT[par]);
  uint16_t* __restrict__ YT = reinterpret_cast<uint16_t*>(a.xT[par ^ 1]);
  const int n = (int)a.n, C = a.C;
  const int ctiles = C / kDBN, tiles = (n / kDBM) * ctiles;
  const int per = (tiles + 7) >> 3;                       // tiles per XCD
  const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  const bool have = tile < tiles;
  const int mt = have ? tile / ctiles : 0, nt = have ? tile % ctiles : 0;
  const int row0 = mt * kDBM, col0 = nt * kDBN;
  const bool work = have && (do_score || a.do_update != 0);

  if (work) {
    f32x16_t P[2][2], Q[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 16; ++r) P[i][j][r] = Q[i][j][r] = 0.0f;
    // two K stages in flight: stage k+1 waits in registers while stage k+2 is loading; the
    // loop is unrolled by two so the two register sets alternate without copies
    DStage r0 = dense_gload2(a.dense_w, XT, n, row0, col0, 0, tid);
    dense_sstore2(As[0], Bs[0], tid, r0);
    r0 = dense_gload2(a.dense_w, XT, n, row0, col0, kDBK, tid);  // n >= 128
    DStage r1;
    __syncthreads();
    for (int k0 = 0; k0 < n; k0 += 2 * kDBK) {  // n % 128 == 0
      // stage k0 from buffer 0; load k0 + 128 (clamped: the last iterations reload a stage into
      // the idle buffer, which keeps the prefetch unconditional); store stage k0 + 64
      r1 = dense_gload2(a.dense_w, XT, n, row0, col0, k0 + 2 * kDBK < n ? k0 + 2 * kDBK : n - kDBK, tid);
      dense_mma_stage(As[0], Bs[0], wm, wn, lo, hi, P, Q);
      dense_sstore2(As[1], Bs[1], tid, r0);
      __syncthreads();
      r0 = dense_gload2(a.dense_w, XT, n, row0, col0, k0 + 3 * kDBK < n ? k0 + 3 * kDBK : n - kDBK, tid);
      dense_mma_stage(As[1], Bs[1], wm, wn, lo, hi, P, Q);
      dense_sstore2(As[0], Bs[0], tid, r1);
      __syncthreads();
    }

    // X_t tile (rows row0.., columns col0..) into LDS with 16-byte loads; row degrees
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = u * 256 + tid, r = e >> 4, c16 = e & 15;
      *reinterpret_cast<uint4*>(&Xs[r][c16 * 8]) =
          *reinterpret_cast<const uint4*>(X + (size_t)(row0 + r) * C + col0 + c16 * 8);
    }
    if (tid < kDBM) s_dw[tid] = a.dw[row0 + tid];
    __syncthreads();
    // element (i, j, r) of this lane: row wm*64 + i*32 + 8*(r/4) + 4*hi + r%4, column wn*64 + j*32 + lo
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int cl = wn * 64 + j * 32 + lo;
      const float eta = a.eta[col0 + cl];
      double colsum = 0.0;  // 32 terms of up to 2^25 each: exact in double
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int vl = wm * 64 + i * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
          const uint32_t hx = Xs[vl][cl];
          const float x = bf2f(hx);
          if (a.do_update) {
            float g = a.cW * P[i][j][r];
            if (a.cD != 0.0f) g = fmaf(a.cD * s_dw[vl], x, g);
            const float y = __builtin_amdgcn_fmed3f(fmaf(eta, g, x), -1.0f, 1.0f);
            Ys[vl][cl] = (uint16_t)(pack_bf16(y, 0.0f) & 0xFFFFu);
          }
          const bool z = (hx & 0x8000u) == 0u && (hx & 0x7FFFu) != 0u;
          colsum += (double)s_dw[vl] - (double)(z ? Q[i][j][r] : -Q[i][j][r]);
        }
      if (do_score) {
        double d = colsum;
        d += __shfl_xor(d, 32);
        if (hi == 0) s_col[wm][cl] = d;
      }
    }
    __syncthreads();
    if (do_score && tid < kDBN) {
      const double v = s_col[0][tid] + s_col[1][tid];
      unsafeAtomicAdd(a.acc + ((size_t)(t & 1) * a.R + (blockIdx.x & (a.R - 1))) * a.B + col0 + tid, v);
    }
    if (a.do_update) {
      // X_t+1 rows and XT_t+1 rows (columns of the tile), 16 bytes per store
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = u * 256 + tid, r = e >> 4, c16 = e & 15;
        *reinterpret_cast<uint4*>(Y + (size_t)(row0 + r) * C + col0 + c16 * 8) =
            *reinterpret_cast<const uint4*>(&Ys[r][c16 * 8]);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = u * 256 + tid, c = e >> 4, v8 = (e & 15) * 8;
        uint32_t w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) w[q] = (uint32_t)Ys[v8 + 2 * q][c] | ((uint32_t)Ys[v8 + 2 * q + 1][c] << 16);
        *reinterpret_cast<uint4*>(YT + (size_t)(col0 + c) * n + row0 + v8) = make_uint4(w[0], w[1], w[2], w[3]);
      }
    }
    if (do_score) {
      // cut bits of X_t, one byte per 8 columns, and the fold of the previous step's improvements
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = u * 256 + tid, r = e >> 4, b = e & 15;
        const uint4 w = *reinterpret_cast<const uint4*>(&Xs[r][b * 8]);
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
        uint32_t byte = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t np = __builtin_bit_cast(uint32_t, nonpos_pair(ws[q]));  // 1 where x <= 0
          byte |= (((np & 1u) ^ 1u) | ((((np >> 16) & 1u) ^ 1u) << 1)) << (2 * q);
        }
        const size_t bi = (size_t)(row0 + r) * a.NBY + (col0 >> 3) + b;
        if (fp >= 0) {
          const uint32_t m = fmask[(col0 >> 3) + b];
          if (m) a.best_bits[bi] = (uint8_t)((a.best_bits[bi] & ~m) | (fbits[bi] & m));
        }
        a.bits[t % 3][bi] = (uint8_t)byte;
      }
    }
  } else if (have && fp >= 0) {
    // a launch that does not score still folds the pending improvements of its tile
    for (int e = tid; e < kDBM * (kDBN / 8); e += 256) {
      const int v = row0 + e / (kDBN / 8);
      const int by = (col0 >> 3) + e % (kDBN / 8);
      const uint32_t m = fmask[by];
      if (m) {
        const size_t bi = (size_t)v * a.NBY + by;
        a.best_bits[bi] = (uint8_t)((a.best_bits[bi] & ~m) | (fbits[bi] & m));
      }
    }
  }
  complete_step(a, t, do_score, cp, s_last);
}

// XT = X^T for the dense path (bfloat16, n x C -> C x n), 64 x 64 tiles through LDS.
__global__ void k_transpose_bf16(const uint16_t* __restrict__ X, uint16_t* __restrict__ XT, int n, int C) {
  __shared__ uint16_t T[64][66];
  const int v0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x) T[i >> 6][i & 63] = X[(size_t)(v0 + (i >> 6)) * C + c0 + (i & 63)];
  __syncthreads();
  for (int i = threadIdx.x; i < 64 * 64; i += blockDim.x) XT[(size_t)(c0 + (i >> 6)) * n + v0 + (i & 63)] = T[i & 63][i >> 6];
}

// Row v: symmetry, zero diagonal, finiteness (flags 2, 1, 4), non-integer weights (16) and a
// weight magnitude sum above 2^24 (32: then W s or d_w could leave the float32 integers);
// d_w(v) in double, stored as float32 (exact when the checks pass).
__global__ void k_dense_validate(const uint16_t* W, int n, float* dw, int* flags) {
  const int v = blockIdx.x;
  double s = 0.0, sa = 0.0;
  int f = 0;
  for (int u = threadIdx.x; u < n; u += blockDim.x) {
    const uint32_t h = W[(size_t)v * n + u];
    const float w = bf2f(h);
    if (!isfinite(w)) f |= 4;
    if (u == v && h != 0u && h != 0x8000u) f |= 1;
    if (W[(size_t)u * n + v] != h) f |= 2;
    if (w != floorf(w)) f |= 16;
    s += (double)w;
    sa += fabs((double)w);
  }
  for (int o = 32; o > 0; o >>= 1) {
    s += __shfl_xor(s, o);
    sa += __shfl_xor(sa, o);
    f |= __shfl_xor(f, o);
  }
  __shared__ double ss[16], sb[16];
  __shared__ int sf[16];
  if ((threadIdx.x & 63) == 0) {
    ss[threadIdx.x >> 6] = s;
    sb[threadIdx.x >> 6] = sa;
    sf[threadIdx.x >> 6] = f;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0, tabs = 0.0;
    int ff = 0;
    for (int i = 0; i < (int)blockDim.x / 64; ++i) {
      tot += ss[i];
      tabs += sb[i];
      ff |= sf[i];
    }
    if (tabs > 16777216.0) ff |= 32;
    dw[v] = (float)tot;
    if (ff) atomicOr(flags, ff);
  }
}

// MOM selects the kernels with a velocity path; they are instantiated only in the
// translation unit of the momentum launcher (step_momentum.hip), so the two halves of the
// step-kernel family compile in parallel.
template <typename T, int VEC, int LL, bool MOM>
hipError_t step_dispatch(const StepArgs& a, int wmode, int grid, hipStream_t s) {
  const dim3 g(grid + a.nextra), b(kThreads);
  if constexpr (MOM) {
    // momentum kernels read the lifted flag at run time
    if (wmode == kUnitW)
      hipLaunchKernelGGL((k_step<T, VEC, LL, kUnitW, -1, true>), g, b, 0, s, a);
    else if (wmode == kPm1W)
      hipLaunchKernelGGL((k_step<T, VEC, LL, kPm1W, -1, true>), g, b, 0, s, a);
    else if (wmode == kIntW)
      hipLaunchKernelGGL((k_step<T, VEC, LL, kIntW, -1, true>), g, b, 0, s, a);
    else
      hipLaunchKernelGGL((k_step<T, VEC, LL, kRealW, -1, true>), g, b, 0, s, a);
    return hipGetLastError();
  } else {
  // rows of one component take the lifted flag (which selects x > 0 or x >= 0 as the side)
  // as a compile-time constant; with l > 1 components the side is always sum >= 0, and
  // 4-value lanes take the kernel without load predicates: the launch runs the largest active
  // count of components, and gathering the zeros of an initialisation with fewer was measured
  // faster than predicating the loads
  constexpr int kOff = LL == 1 ? 0 : -1, kOn = LL == 1 ? 1 : -1;
  const bool on = LL == 1 && a.lifted;
  if constexpr (LL > 1 && LL <= 4 && (VEC == 4 || VEC == 2)) {
    if (wmode == kUnitW)
      hipLaunchKernelGGL((k_step<T, VEC, LL, kUnitW, -1, false, true>), g, b, 0, s, a);
    else if (wmode == kPm1W)
      hipLaunchKernelGGL((k_step<T, VEC, LL, kPm1W, -1, false, true>), g, b, 0, s, a);
    else if (wmode == kIntW)
      hipLaunchKernelGGL((k_step<T, VEC, LL, kIntW, -1, false, true>), g, b, 0, s, a);
    else
      hipLaunchKernelGGL((k_step<T, VEC, LL, kRealW, -1, false, true>), g, b, 0, s, a);
  } else {
    if (wmode == kUnitW) {
      if (on)
        hipLaunchKernelGGL((k_step<T, VEC, LL, kUnitW, kOn, false>), g, b, 0, s, a);
      else
        hipLaunchKernelGGL((k_step<T, VEC, LL, kUnitW, kOff, false>), g, b, 0, s, a);
    } else if (wmode == kPm1W) {
      if (on)
        hipLaunchKernelGGL((k_step<T, VEC, LL, kPm1W, kOn, false>), g, b, 0, s, a);
      else
        hipLaunchKernelGGL((k_step<T, VEC, LL, kPm1W, kOff, false>), g, b, 0, s, a);
    } else if (wmode == kIntW) {
      if (on)
        hipLaunchKernelGGL((k_step<T, VEC, LL, kIntW, kOn, false>), g, b, 0, s, a);
      else
        hipLaunchKernelGGL((k_step<T, VEC, LL, kIntW, kOff, false>), g, b, 0, s, a);
    } else {
      if (on)
        hipLaunchKernelGGL((k_step<T, VEC, LL, kRealW, kOn, false>), g, b, 0, s, a);
      else
        hipLaunchKernelGGL((k_step<T, VEC, LL, kRealW, kOff, false>), g, b, 0, s, a);
    }
  }
  return hipGetLastError();
  }
}

// All component counts for float32 and one-element lanes; bfloat16 runs unlifted rows 8 or
// 4 values per lane and lifted rows (l > 1) 4 values per lane; 2-value lanes (float32 by
// default, bfloat16 as a tuned choice) run rows of 2 to 4 components here and of 5 to 8 in
// step_wide.hip, without momentum (launch_step maps the rest to 4-value lanes).
template <typename T, int VEC, bool MOM>
hipError_t step_dispatch_l(const StepArgs& a, int wmode, int grid, hipStream_t s) {
  constexpr bool bf_wide = sizeof(T) == 2 && VEC == 8;
  constexpr bool pair = VEC == 2;
  if constexpr (pair) {
    if (MOM || a.L == 1) return hipErrorInvalidValue;
  } else {
    if (a.L == 1) return step_dispatch<T, VEC, 1, MOM>(a, wmode, grid, s);
  }
  if constexpr (!bf_wide) {
    switch (a.L) {
      case 2: return step_dispatch<T, VEC, 2, MOM>(a, wmode, grid, s);
      case 3: return step_dispatch<T, VEC, 3, MOM>(a, wmode, grid, s);
      case 4: return step_dispatch<T, VEC, 4, MOM>(a, wmode, grid, s);
      default: break;
    }
  }
  return hipErrorInvalidValue;
}

inline int step_weight_mode(const StepArgs& a) {
  return a.w == nullptr ? kUnitW : (a.pm1 ? kPm1W : (a.intw ? kIntW : kRealW));
}

template <bool MOM>
hipError_t launch_step_impl(const StepArgs& a, int dtype, int vec, int grid, hipStream_t s) {
  const int wmode = step_weight_mode(a);
  if (dtype == 0) {
    if (vec == 4) return step_dispatch_l<float, 4, MOM>(a, wmode, grid, s);
    if constexpr (!MOM)
      if (vec == 2) return step_dispatch_l<float, 2, MOM>(a, wmode, grid, s);
    if (vec == 1) return step_dispatch_l<float, 1, MOM>(a, wmode, grid, s);
  } else {
    if (vec == 8) return step_dispatch_l<uint16_t, 8, MOM>(a, wmode, grid, s);
    if (vec == 4) return step_dispatch_l<uint16_t, 4, MOM>(a, wmode, grid, s);
    if constexpr (!MOM)
      if (vec == 2) return step_dispatch_l<uint16_t, 2, MOM>(a, wmode, grid, s);
    if (vec == 1) return step_dispatch_l<uint16_t, 1, MOM>(a, wmode, grid, s);
  }
  return hipErrorInvalidValue;
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
    if (wk != floorf(wk) || fabsf(wk) > 1024.0f) f |= 16;
    if (fabsf(wk) != 1.0f) f |= 32;
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

// ------------------------------------------------------------------ slot list
// Row v's own slot at row_ptr[v] + v (index with the top bit set; weighted degree as its
// weight), one thread per row.
__global__ void k_slots_self(long long n, const int* rp, const float* dw, int* slots, float* sw) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const long long p = (long long)rp[v] + v;
  slots[p] = (int)((unsigned)v | 0x80000000u);
  if (sw) sw[p] = dw[v];
}

// Edge e of row v (the last row with row_ptr[v] <= e) goes to slot e + v + 1, one thread
// per edge.
__global__ void k_slots_edges(long long n, long long nnz, const int* rp, const int* ci, const float* w, int* slots,
                              float* sw) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  long long lo = 0, hi = n;  // rp[lo] <= e < rp[hi]
  while (hi - lo > 1) {
    const long long mid = (lo + hi) >> 1;
    if (rp[mid] <= e) lo = mid; else hi = mid;
  }
  const long long p = e + lo + 1;
  slots[p] = ci[e];
  if (sw) sw[p] = w[e];
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
  if (i < 2LL * a.G * a.NBY) a.mask[i] = 0;
  if (i < 8) a.ctrl->xticket[i][0] = 0u;
  if (i == 0) {
    a.ctrl->ticket = 0u;
    a.ctrl->score_every = score_every;
    a.ctrl->t = 0;
    a.ctrl->cpend = -1;
    a.ctrl->fpend = -1;
    a.ctrl->drain[0] = -1;
    a.ctrl->drain[1] = -1;
  }
}

// First half of a drain: completes the pending scored step (if any) and records the steps
// whose improvements the merge folds, older first.
__global__ __launch_bounds__(256) void k_complete(StepArgs a) {
  const long long cp = a.ctrl->cpend;
  if (cp >= 0) finish_scores(a, cp, blockIdx.x, gridDim.x);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.ctrl->drain[0] = a.ctrl->fpend;
    a.ctrl->drain[1] = cp;
  }
}

// Second half of a drain: folds the improvements of the recorded steps into best_bits, in
// order, and clears the pending marks (idempotent until the bit slots are reused).
__global__ void k_merge(StepArgs a, long long n, const int* goff) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    a.ctrl->cpend = -1;
    a.ctrl->fpend = -1;
  }
  if (i >= n * a.NBY) return;
  const long long row = i / a.NBY;
  const int by = (int)(i % a.NBY);
  int lo = 0, hi = a.G;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (goff[mid] <= row) lo = mid; else hi = mid;
  }
  for (int k = 0; k < 2; ++k) {
    const long long s = a.ctrl->drain[k];
    if (s < 0) continue;
    const uint32_t m = a.mask[(size_t)(s & 1) * a.G * a.NBY + lo * a.NBY + by];
    if (m) {
      const uint32_t bits = a.bits[s % 3][i];
      const uint32_t bb = a.best_bits[i];
      a.best_bits[i] = (uint8_t)((bb & ~m) | (bits & m));
    }
  }
}

__global__ void k_fill(float* p, int n, float v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Zeroes n 16-bit words (grid-stride).
__global__ void k_zero16(uint16_t* p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0;
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
  } else if (a.kind == 3 || a.kind == 5) {  // IDI (kind 5: times a learned magnitude)
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
  if (a.kind == 5) h *= (double)a.magnitude[v];
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

#ifndef DECO_KERNELS_ONLY_TU  // the host launchers live in this translation unit only
int native_vec(int dtype, int L) { return dtype == 0 ? (L >= 2 && L <= 8 ? 2 : 4) : (L == 1 ? 8 : 4); }

hipError_t launch_dense_transpose(const void* X, void* XT, long long n, int C, hipStream_t s) {
  hipLaunchKernelGGL(k_transpose_bf16, dim3((unsigned)(n / 64), (unsigned)(C / 64)), dim3(256), 0, s,
                     reinterpret_cast<const uint16_t*>(X), reinterpret_cast<uint16_t*>(XT), (int)n, C);
  return hipGetLastError();
}

hipError_t launch_dense_step(const StepArgs& a, hipStream_t s) {
  const int tiles = (int)(a.n / kDBM) * (a.C / kDBN);
  const int grid = 8 * ((tiles + 7) / 8);
  hipLaunchKernelGGL(k_dense_step, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_dense_validate(const uint16_t* W, int n, float* dw, int* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_dense_validate, dim3(n), dim3(256), 0, s, W, n, dw, flags);
  return hipGetLastError();
}

hipError_t launch_step(const StepArgs& a, int dtype, int vec, int grid, hipStream_t s) {
  if (vec == 2 && (a.L == 1 || a.vel != nullptr)) {
    // a tile of Wc 2-value lanes is the same tile as Wc/2 4-value lanes (the work list
    // depends on the tile only): run the kernels of 4-value lanes on it
    if (a.Wc < 2) return hipErrorInvalidValue;
    StepArgs b = a;
    b.Wc = a.Wc / 2;
    return launch_step(b, dtype, 4, grid, s);
  }
  if (a.L > 4) return launch_step_wide(a, dtype, vec, grid, s);
  if (a.vel != nullptr) return launch_step_momentum(a, dtype, vec, grid, s);
  return launch_step_impl<false>(a, dtype, vec, grid, s);
}

hipError_t launch_validate(long long n, const int* rp, const int* ci, const float* w,
                           const int* goff, int G, float* dw, int* flags, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_validate, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, ci, w, goff, G,
                     dw, flags);
  return hipGetLastError();
}

hipError_t launch_build_slots(long long n, long long nnz, const int* rp, const int* ci, const float* w,
                              const float* dw, int* slots, float* sw, hipStream_t s) {
  hipLaunchKernelGGL(k_slots_self, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, rp, dw, slots, w ? sw : nullptr);
  if (nnz > 0)
    hipLaunchKernelGGL(k_slots_edges, dim3(blocks_for(nnz, 256)), dim3(256), 0, s, n, nnz, rp, ci, w, slots,
                       w ? sw : nullptr);
  return hipGetLastError();
}

hipError_t launch_reset(StepArgs a, double* acc_all, long long acc_count, int score_every,
                        hipStream_t s) {
  long long m = acc_count;
  const long long GB = (long long)a.G * a.B;
  if (GB > m) m = GB;
  if (2LL * a.G * a.NBY > m) m = 2LL * a.G * a.NBY;
  if (m < 1) m = 1;
  hipLaunchKernelGGL(k_reset, dim3(blocks_for(m, 256)), dim3(256), 0, s, a, acc_all, acc_count,
                     score_every);
  return hipGetLastError();
}

int completion_blocks(long long GB) {
  const long long b = (GB + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 64 ? 64 : b));
}

hipError_t launch_drain(StepArgs a, long long n, const int* goff, hipStream_t s) {
  hipLaunchKernelGGL(k_complete, dim3(completion_blocks((long long)a.G * a.B)), dim3(256), 0, s, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_merge(a, n, goff, s);
}

hipError_t launch_merge(StepArgs a, long long n, const int* goff, hipStream_t s) {
  const long long m = n * a.NBY;
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_merge, dim3(blocks_for(m, 256)), dim3(256), 0, s, a, n, goff);
  return hipGetLastError();
}

// Sides of a batch with many components per initialisation (l above kMaxL, run as an
// unlifted handle over the l B columns plus a lifted l = 1 handle over the B sums): S[v, b] =
// sum_{i<l} X[v, i B + b] in float32, component order i = 0..l-1 (the lifted rounding of
// Sec. 3.2 takes its sign), stored in the storage type (round to nearest even keeps the
// sign; -0 and +0 both give side 1). With control blocks the iterate is x[tx & 1] and the sums
// go to s[ts & 1] (tx, ts: the two handles' step counters, read on the device so a captured
// graph replays correctly); without them x0 and s0 are used.
__global__ void k_sides(const void* x0, const void* x1, void* s0, void* s1, const DevCtrl* cx, const DevCtrl* cs,
                        long long n, int B, int l, int dtype) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * B) return;
  const long long v = i / B;
  const int b = (int)(i % B);
  const void* X = (cx && (cx->t & 1)) ? x1 : x0;
  void* S = (cs && (cs->t & 1)) ? s1 : s0;
  const size_t base = (size_t)v * B * l + b;
  float sum = 0.0f;
  if (dtype == 0) {
    const float* x = reinterpret_cast<const float*>(X) + base;
    for (int c = 0; c < l; ++c) sum = sum + x[(size_t)c * B];
    reinterpret_cast<float*>(S)[i] = sum;
  } else {
    const uint16_t* x = reinterpret_cast<const uint16_t*>(X) + base;
    for (int c = 0; c < l; ++c) sum = sum + bf2f(x[(size_t)c * B]);
    reinterpret_cast<uint16_t*>(S)[i] = (uint16_t)(pack_bf16(sum, 0.0f) & 0xFFFFu);
  }
}

hipError_t launch_sides(const void* x0, const void* x1, void* s0, void* s1, const DevCtrl* cx, const DevCtrl* cs,
                        long long n, int B, int l, int dtype, hipStream_t s) {
  const long long m = n * B;
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sides, dim3(blocks_for(m, 256)), dim3(256), 0, s, x0, x1, s0, s1, cx, cs, n, B, l, dtype);
  return hipGetLastError();
}

hipError_t launch_fill_eta(float* eta, int B, float v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(B, 256)), dim3(256), 0, s, eta, B, v);
  return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  const long long n = (long long)(bytes / 2);
  if (n <= 0) return hipSuccess;
  const long long blocks = (n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192;
  hipLaunchKernelGGL(k_zero16, dim3((unsigned)blocks), dim3(256), 0, s, reinterpret_cast<uint16_t*>(p), n);
  return hipGetLastError();
}

hipError_t launch_init(const InitArgs& a, hipStream_t s) {
  const long long m = a.n * a.C;
  if (m <= 0) return hipSuccess;
  if (a.kind == 3 || a.kind == 5) {
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

#endif  // DECO_KERNELS_ONLY_TU

}  // namespace deco
