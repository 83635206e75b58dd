// Host side of the DECO library: the C ABI of include/deco.h.
//
// A handle binds a caller-owned graph, iterate X and workspace. deco_init validates the
// graph on the device, keeps a host copy of row_ptr and builds the work schedule: rows are
// cut into items of bounded edge count, every item is paired with each initialisation tile,
// and items are grouped per XCD (workgroup i runs on XCD i % 8), either by contiguous row
// ranges or by initialisation tile, so that one XCD's L2 keeps serving the gathers of the
// rows / tile it owns. deco_autotune times a set of candidate schedules on the device.
// deco_solve is the host loop of pDECO (Alg. 3) with the evolutionary search of Sec. 4.3.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/deco.h"
#include "internal.h"

using namespace deco;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMinTile = 64;       // narrowest initialisation tile when B >= 64 (unlifted)
constexpr int kMinTileLifted = 16; // lifted rows carry l values per initialisation: narrower tiles

// Narrowest initialisation tile of a handle: unlifted tiles of at least 64 when 64 divides B
// (narrower ones multiply the per-slot work without shrinking it); lifted rows hold l values
// per initialisation, so tiles down to 16 keep a lane's gathers wide and let each XCD own a
// tile small enough for its L2.
int min_tile(int B, int l) {
  if (l >= 2) return B % kMinTileLifted == 0 ? kMinTileLifted : (B >= 8 ? 8 : B);
  return B % kMinTile == 0 ? kMinTile : (B >= 8 ? 8 : B);
}
constexpr int kMinItemSlots = 128; // smallest nnz_per_item
constexpr int kMaxBlocksPerXcd = 4096;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Schedule {
  int vec = 4;
  int Wc = 1;         // lanes per row team
  int dlong = 64;     // rows with more neighbours get a work item of their own
  int rows_per_item = 256;
  int nnz_per_item = 2048;
  int xcd_mode = 0;   // 0 rows per XCD, 1 initialisation tiles per XCD
  int blocks_per_xcd = 128;
  int grid = 0;
  int nitems = 0;
  std::vector<int4> items;  // {first row, end row, graph, tile | long << 16}
  int seg[9] = {0};
  // resident schedule (resident.hip): rbt columns of a graph's rows per workgroup, all steps of
  // a call in one launch; 0 = the step kernel
  int rbt = 0;
  int rmax_rows = 0;
  std::vector<int4> ritems;  // {graph, first row, end row, first column}
  std::vector<int4> rgs;     // per graph: {stream offset, slots per thread, slots, first slot}
};

// LDS a workgroup may use (queried once; gfx950 allows up to 160 KB per workgroup).
int lds_limit() {
  static int v = [] {
    int dev = 0, bytes = 65536;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      bytes = 65536;
    return bytes;
  }();
  return v;
}

// LDS left for the resident kernel's dynamic part (its static arrays take at most ~2 KB).
constexpr int kResidentStaticLds = 2048;

struct Layout {
  size_t xalt, bits0, bits1, bits2, best_bits, mask, acc, cur_cut, best_cut, best_step, ctrl, dw, eta,
      slots, sw, items, seg, goff, thr, delta, l_active, flags, xt0, xt1, ritems, rstream, rwstream, rgs, rbest, rimp,
      total;
  long long items_cap;
  long long rstream_cap;  // ints of the resident schedule's slot streams
  int R;
};

int elem_size(int dtype) { return dtype == DECO_BF16 ? 2 : 4; }
int nby_of(int B) { return (B + 7) / 8; }

bool supported_B(int B) { return B == 1 || B == 2 || B == 4 || (B > 0 && B % 8 == 0); }

int vec_for(int dtype, int B, int L) { return (B % 8 == 0) ? native_vec(dtype, L) : 1; }

// Largest lane count per row team (power of two, <= 64) whose tile divides B and holds at
// most 256 initialisations.
int max_wc(int vec, int B) {
  int wc = 1;
  while (wc * 2 <= 64 && wc * 2 * vec <= 256 && B % (wc * 2 * vec) == 0) wc *= 2;
  return wc;
}

Layout layout_for(long long n, long long nnz, int G, const deco_params* p, bool weighted, bool dense = false) {
  Layout L{};
  const int C = p->l * p->B;
  const int NBY = nby_of(p->B);
  const int vec = vec_for(p->x_dtype, p->B, p->l);
  // initialisation tiles are at least kMinTile wide when kMinTile divides B, else at least
  // 8 wide (or the whole of B < 8). A chunk
  // and the row after it hold more than nnz_per_item >= kMinItemSlots slots, or the chunk
  // holds kRmax rows, or ends a graph, or precedes a row isolated by the neighbour limit
  // (at least 17 neighbours)
  const long long nbt_max = std::max(1, p->B / min_tile(p->B, p->l));
  (void)vec;
  L.R = G >= 16 ? 1 : 16;
  L.items_cap = nbt_max * (2 * (n + nnz) / kMinItemSlots + n / kRmax + 2 * (nnz / 17) + (long long)G + 8);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return o;
  };
  L.xalt = take((size_t)n * C * elem_size(p->x_dtype));
  L.bits0 = take((size_t)n * NBY);
  L.bits1 = take((size_t)n * NBY);
  L.bits2 = take((size_t)n * NBY);
  L.best_bits = take((size_t)n * NBY);
  L.mask = take(2 * (size_t)G * NBY);
  L.acc = take(2 * sizeof(double) * (size_t)L.R * G * p->B);
  L.cur_cut = take(sizeof(double) * (size_t)G * p->B);
  L.best_cut = take(sizeof(double) * (size_t)G * p->B);
  L.best_step = take(sizeof(int) * (size_t)G * p->B);
  L.ctrl = take(sizeof(DevCtrl));
  L.dw = take(sizeof(float) * (size_t)n);
  L.eta = take(sizeof(float) * (size_t)p->B);
  L.slots = take(sizeof(int) * (size_t)(n + nnz));
  L.sw = take(weighted ? sizeof(float) * (size_t)(n + nnz) : 0);
  L.items = take(2 * sizeof(int4) * (size_t)L.items_cap);
  L.seg = take(sizeof(int) * 16);
  L.goff = take(sizeof(int) * (size_t)(G + 1));
  L.thr = take(sizeof(double) * (size_t)G);
  L.delta = take(sizeof(int) * (size_t)G);
  L.l_active = take(sizeof(int) * (size_t)p->B);
  L.flags = take(sizeof(int) * 4);
  // dense path: transposed ping-pong iterates
  L.xt0 = take(dense ? (size_t)n * C * elem_size(p->x_dtype) : 0);
  L.xt1 = take(dense ? (size_t)n * C * elem_size(p->x_dtype) : 0);
  // resident schedule: one work item per (graph, column) at most
  L.ritems = take(dense || p->l != 1 ? 0 : sizeof(int4) * (size_t)G * p->B);
  // and the graphs' slot lists split into equal shares per thread, interleaved (each graph's
  // shares are rounded up to 4 slots, after 4 ints of header, for at most 1024 threads)
  L.rstream_cap = dense || p->l != 1 ? 0 : (n + nnz) + 8LL * 1024 * G;
  L.rstream = take(sizeof(int) * (size_t)L.rstream_cap);
  L.rwstream = take(weighted ? sizeof(float) * (size_t)L.rstream_cap : 0);
  L.rgs = take(dense || p->l != 1 ? 0 : sizeof(int4) * (size_t)G);
  // best sides of resident tiles narrower than a byte of best_bits, and their improved flags
  L.rbest = take(dense || p->l != 1 ? 0 : (size_t)n * p->B);
  L.rimp = take(dense || p->l != 1 ? 0 : (size_t)G * p->B);
  L.total = off;
  return L;
}

}  // namespace

struct deco_handle {
  deco_graph g{};
  deco_params p{};
  hipStream_t stream = nullptr;
  long long n = 0, nnz = 0;
  int G = 1, C = 1, NBY = 1, R = 1, dtype = 0;
  bool unit = true;
  bool dense = false;  // dense-matrix (MFMA) path
  bool poisoned = false;
  Layout lay{};
  char* ws = nullptr;
  void* X = nullptr;
  StepArgs args{};
  Schedule sched;
  std::vector<int> rp_host;
  std::vector<int> goff_host;
  std::vector<int> lact_host;  // host copy of the step kernel's active-component counts
  // More than kMaxL components per initialisation: the iterates live in cx, an unlifted handle
  // over the l B columns (the lifted update acts column by column, Sec. 3.2), and the scores in
  // cs, a lifted l = 1 handle over the B component sums (its step size is 0, so a step only
  // scores and advances); k_sides refreshes cs's iterate from cx's before every scoring.
  deco_handle* cx = nullptr;
  deco_handle* cs = nullptr;
  char* sbuf = nullptr;  // n x B sums for starts
  long long t_host = 0;
  double* trace = nullptr;
  int trace_cap = 0;
  std::map<int, hipGraphExec_t> graphs;
};

namespace {

deco_status poison(deco_handle* h, hipError_t e) {
  if (e == hipSuccess) return DECO_OK;
  if (h) h->poisoned = true;
  return DECO_E_DEVICE;
}

#define HIP_TRY(h, expr)                        \
  do {                                          \
    hipError_t e__ = (expr);                    \
    if (e__ != hipSuccess) return poison((h), e__); \
  } while (0)

// Split each graph's rows into work chunks of about nnz_per_item slots (edges plus rows):
// a chunk closes before the row that would take it past nnz_per_item slots or kRmax /
// rows_per_item rows. A row of more than nnz_per_item slots or more than dlong neighbours
// is a chunk of its own, flagged in .w as a long row when its slots exceed kEmax.
std::vector<int4> row_chunks(const std::vector<int>& rp, const std::vector<int>& goff, int rows_per_item,
                             int nnz_per_item, int dlong) {
  std::vector<int4> ch;
  const int G = (int)goff.size() - 1;
  const int rmax = std::min(rows_per_item, kRmax);
  for (int g = 0; g < G; ++g) {
    int start = -1;
    long long e = 0;
    for (int r = goff[g]; r < goff[g + 1]; ++r) {
      const int d = rp[r + 1] - rp[r] + 1;  // slots of the row
      if (d - 1 > dlong || d > nnz_per_item) {
        if (start >= 0) ch.push_back(make_int4(start, r, g, 0));
        start = -1;
        ch.push_back(make_int4(r, r + 1, g, d > kEmax ? 1 << 16 : 0));
        continue;
      }
      if (start >= 0 && (r - start >= rmax || e + d > nnz_per_item)) {
        ch.push_back(make_int4(start, r, g, 0));
        start = -1;
      }
      if (start < 0) {
        start = r;
        e = 0;
      }
      e += d;
    }
    if (start >= 0) ch.push_back(make_int4(start, goff[g + 1], g, 0));
  }
  return ch;
}

// Cut the chunk list into 'parts' contiguous groups of about equal weight (rows + edges).
std::vector<int> balance(const std::vector<int4>& ch, const std::vector<int>& rp, int parts) {
  std::vector<int> cut(parts + 1, 0);
  long long total = 0;
  for (auto& c : ch) total += (c.y - c.x) + (rp[c.y] - rp[c.x]);
  long long acc = 0;
  int p = 1;
  for (size_t i = 0; i < ch.size() && p < parts; ++i) {
    acc += (ch[i].y - ch[i].x) + (rp[ch[i].y] - rp[ch[i].x]);
    while (p < parts && acc * parts >= total * p) cut[p++] = (int)i + 1;
  }
  while (p < parts) cut[p++] = (int)ch.size();
  cut[parts] = (int)ch.size();
  return cut;
}

bool build_schedule(deco_handle* h, Schedule& s) {
  const int B = h->p.B;
  if (s.rbt > 0) {
    // every graph's rows times rbt columns, two buffers, in one workgroup's LDS
    if (h->dense || h->p.l != 1 || B % s.rbt != 0 || (s.rbt & (s.rbt - 1)) || s.rbt > 16) return false;
    const std::vector<int>& goff = h->goff_host;
    int maxr = 1;
    for (int g = 0; g < h->G; ++g) maxr = std::max(maxr, goff[g + 1] - goff[g]);
    if (resident_lds_bytes(maxr, s.rbt, h->dtype) + kResidentStaticLds > (size_t)lds_limit()) return false;
    // largest graphs first: the dispatcher hands the long items out first
    std::vector<int> order(h->G);
    for (int g = 0; g < h->G; ++g) order[g] = g;
    const std::vector<int>& rp = h->rp_host;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return (long long)(rp[goff[x + 1]] - rp[goff[x]]) + (goff[x + 1] - goff[x]) >
             (long long)(rp[goff[y + 1]] - rp[goff[y]]) + (goff[y + 1] - goff[y]);
    });
    s.ritems.clear();
    for (int g : order)
      for (int c0 = 0; c0 < B; c0 += s.rbt) s.ritems.push_back(make_int4(g, goff[g], goff[g + 1], c0));
    s.rmax_rows = maxr;
    // equal shares of each graph's slots per thread, rounded up to 4 (one 16-byte load)
    const int nt = resident_threads(s.rbt);
    s.rgs.assign(h->G, make_int4(0, 0, 0, 0));
    long long soff = 0;
    for (int gi = 0; gi < h->G; ++gi) {
      const long long E = (long long)(rp[goff[gi + 1]] - rp[goff[gi]]) + (goff[gi + 1] - goff[gi]);
      const long long per = ((E + nt - 1) / nt + 3) / 4 * 4;
      s.rgs[gi] = make_int4((int)soff, (int)per, (int)E, rp[goff[gi]] + goff[gi]);
      soff += (4 + per) * nt;  // 4 ints of header per thread, then its slots
    }
    if (soff > h->lay.rstream_cap) return false;
    // the step kernel's work list is built too: score-only passes and momentum steps use it
  }
  const int Bt = s.Wc * s.vec;
  if (Bt <= 0 || Bt > 256 || B % Bt != 0 || (B >= 8 && Bt % 8 != 0)) return false;
  if (B >= 8 && Bt < min_tile(B, h->p.l)) return false;
  if (s.Wc > 64) return false;
  if (s.dlong < 16 || s.nnz_per_item < kMinItemSlots || s.nnz_per_item > kEmax) return false;
  const int nbt = B / Bt;
  auto ch = row_chunks(h->rp_host, h->goff_host, s.rows_per_item, s.nnz_per_item, s.dlong);
  std::vector<int4> items;
  int seg[9];
  const bool tiles = s.xcd_mode == 1 && nbt >= 2 && (nbt >= 8 || 8 % nbt == 0);
  if (!tiles) {
    auto cut = balance(ch, h->rp_host, 8);
    for (int x = 0; x < 8; ++x) {
      seg[x] = (int)items.size();
      for (int bt = 0; bt < nbt; ++bt)
        for (int i = cut[x]; i < cut[x + 1]; ++i) items.push_back(make_int4(ch[i].x, ch[i].y, ch[i].z, ch[i].w | bt));
    }
  } else if (nbt >= 8) {
    for (int x = 0; x < 8; ++x) {
      seg[x] = (int)items.size();
      for (int bt = x; bt < nbt; bt += 8)
        for (auto& c : ch) items.push_back(make_int4(c.x, c.y, c.z, c.w | bt));
    }
  } else {
    const int parts = 8 / nbt;
    auto cut = balance(ch, h->rp_host, parts);
    for (int x = 0; x < 8; ++x) {
      seg[x] = (int)items.size();
      const int bt = x % nbt, part = x / nbt;
      for (int i = cut[part]; i < cut[part + 1]; ++i) items.push_back(make_int4(ch[i].x, ch[i].y, ch[i].z, ch[i].w | bt));
    }
  }
  seg[8] = (int)items.size();
  if ((long long)items.size() > h->lay.items_cap) return false;
  int maxper = 1;
  for (int x = 0; x < 8; ++x) maxper = std::max(maxper, seg[x + 1] - seg[x]);
  s.grid = 8 * std::min(s.blocks_per_xcd, maxper);
  s.nitems = (int)items.size();
  s.items = std::move(items);
  std::memcpy(s.seg, seg, sizeof(seg));
  return true;
}

deco_status upload_schedule(deco_handle* h) {
  char* ws = h->ws;
  if (h->sched.rbt > 0) {
    HIP_TRY(h, hipMemcpyAsync(ws + h->lay.ritems, h->sched.ritems.data(), sizeof(int4) * h->sched.ritems.size(),
                              hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, hipMemcpyAsync(ws + h->lay.rgs, h->sched.rgs.data(), sizeof(int4) * h->sched.rgs.size(),
                              hipMemcpyHostToDevice, h->stream));
    HIP_TRY(h, build_resident_stream(h->n + h->nnz, h->G, h->sched.rbt, reinterpret_cast<const int4*>(ws + h->lay.rgs),
                                     reinterpret_cast<const int*>(ws + h->lay.goff), h->args.rp, h->args.slots,
                                     h->args.sw,
                                     reinterpret_cast<int*>(ws + h->lay.rstream),
                                     h->args.sw ? reinterpret_cast<float*>(ws + h->lay.rwstream) : nullptr,
                                     h->stream));
    HIP_TRY(h, prepare_resident(h->args, h->dtype, h->sched.rbt, h->sched.rmax_rows));
  }
  // device form: {x, y, first slot, end slot}, {graph, tile, long-row flag, 0}
  const std::vector<int>& rp = h->rp_host;
  std::vector<int4> dev(2 * h->sched.items.size());
  for (size_t i = 0; i < h->sched.items.size(); ++i) {
    const int4 c = h->sched.items[i];
    dev[2 * i] = make_int4(c.x, c.y, rp[c.x] + c.x, rp[c.y] + c.y);
    dev[2 * i + 1] = make_int4(c.z, c.w & 0xFFFF, c.w >> 16, 0);
  }
  HIP_TRY(h, hipMemcpyAsync(ws + h->lay.items, dev.data(), sizeof(int4) * dev.size(), hipMemcpyHostToDevice,
                            h->stream));
  HIP_TRY(h, hipMemcpyAsync(ws + h->lay.seg, h->sched.seg, sizeof(int) * 9, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  h->args.Wc = h->sched.Wc;
  for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
  h->graphs.clear();
  return DECO_OK;
}

// Slots one row team gathers per window (the kernel's window for this lane width and l).
int window_slots(int vec, int L, int dtype) {
  const int loads = vec == 1 ? 32 : (L == 1 ? (vec * elem_size(dtype) >= 16 ? 12 : 16) : 8);
  return std::max(1, loads / L);
}

Schedule default_schedule(deco_handle* h) {
  Schedule s;
  // lanes of several elements address rows with 32-bit offsets: n < 2^24 and n * C < 2^32
  const bool small = h->n < (1LL << 24) && (unsigned long long)h->n * h->C < (1ULL << 32);
  s.vec = small ? vec_for(h->dtype, h->p.B, h->p.l) : 1;
  s.Wc = max_wc(s.vec, h->p.B);
  // lifted rows: half-width tiles (twice the teams) when the tile stays wide enough
  if (h->p.l > 1 && s.Wc > 1) {
    const int bt = (s.Wc / 2) * s.vec;
    if (bt >= std::max(min_tile(h->p.B, h->p.l), 8) && bt % 8 == 0) s.Wc /= 2;
  }
  s.dlong = 1 << 30;  // rows are isolated only by the item size
  s.xcd_mode = 0;
  // one item per workgroup (the dispatcher balances the rest); items large enough to give
  // every team of a workgroup a window, and about as many as workgroups fit on the chip at
  // once (256 CUs x 3)
  s.blocks_per_xcd = kMaxBlocksPerXcd;
  const long long slots = h->nnz + h->n;
  const long long teams = 256 / s.Wc;
  const long long per = std::max<long long>(teams * window_slots(s.vec, h->p.l, h->dtype), (slots + 767) / 768);
  s.nnz_per_item = (int)std::max<long long>(kMinItemSlots, std::min<long long>(kEmax, per));
  s.rows_per_item = kRmax;
  return s;
}

bool schedule_cached(const deco_handle* h);

std::mutex g_cache_mu;
std::map<std::tuple<long long, long long, int, int, int, int, int>, Schedule> g_cache;

std::tuple<long long, long long, int, int, int, int, int> cache_key(const deco_handle* h) {
  return std::make_tuple(h->n, h->nnz, h->G, h->p.B, h->p.l, h->dtype, h->unit ? 1 : 0);
}

bool schedule_cached(const deco_handle* h) {
  if (h->cx) return schedule_cached(h->cx) && schedule_cached(h->cs);
  std::lock_guard<std::mutex> lk(g_cache_mu);
  return g_cache.count(cache_key(h)) != 0;
}

deco_status check_graph_args(const deco_graph* g) {
  if (!g || g->n < 1 || g->nnz < 0 || !g->row_ptr || (g->nnz > 0 && !g->col_idx)) return DECO_E_INVAL;
  if (g->num_graphs < 1 || (g->num_graphs > 1 && !g->graph_row_offset)) return DECO_E_INVAL;
  if (g->n + g->nnz >= (1LL << 31) - 1) return DECO_E_UNSUPPORTED;  // slot indices are int32
  if (g->num_graphs > g->n) return DECO_E_INVAL;
  return DECO_OK;
}

deco_status check_params(const deco_params* p) {
  if (!p) return DECO_E_INVAL;
  if (p->B < 1 || p->l < 1 || p->score_every < 1) return DECO_E_INVAL;
  if (p->x_dtype != DECO_F32 && p->x_dtype != DECO_BF16) return DECO_E_INVAL;
  if (p->grad_form != DECO_GRAD_CUT && p->grad_form != DECO_GRAD_LAPLACIAN) return DECO_E_INVAL;
  if (!p->lifted && p->l != 1) return DECO_E_INVAL;
  if (!std::isfinite(p->eta)) return DECO_E_NONFINITE;
  if (!supported_B(p->B) || (long long)p->l * p->B >= (1LL << 24)) return DECO_E_UNSUPPORTED;
  return DECO_OK;
}

deco_status launch_steps(deco_handle* h, int steps, int do_update, int force) {
  StepArgs a = h->args;
  a.do_update = do_update;
  a.force_score = force;
  if (h->sched.rbt > 0 && do_update && !force && a.vel == nullptr && !h->dense) {
    const hipError_t e =
        launch_resident(a, h->dtype, h->sched.rbt, reinterpret_cast<const int4*>(h->ws + h->lay.ritems),
                        (int)h->sched.ritems.size(), reinterpret_cast<const int4*>(h->ws + h->lay.rgs),
                        reinterpret_cast<const int*>(h->ws + h->lay.rstream),
                        a.sw ? reinterpret_cast<const float*>(h->ws + h->lay.rwstream) : nullptr,
                        reinterpret_cast<uint8_t*>(h->ws + h->lay.rbest), reinterpret_cast<uint8_t*>(h->ws + h->lay.rimp),
                        reinterpret_cast<const int*>(h->ws + h->lay.goff), h->sched.rmax_rows, steps, h->stream);
    return e == hipSuccess ? DECO_OK : poison(h, e);
  }
  for (int s = 0; s < steps; ++s) {
    const hipError_t e = h->dense ? launch_dense_step(a, h->stream)
                                  : launch_step(a, h->dtype, h->sched.vec, h->sched.grid, h->stream);
    if (e != hipSuccess) return poison(h, e);
  }
  return DECO_OK;
}

// One step of a many-component handle: sums of X_t into the score handle, a scoring step of
// the score handle (step size 0: it scores X_t's sides and advances), the step of the iterates.
deco_status wide_launch_steps(deco_handle* h, int steps) {
  for (int t = 0; t < steps; ++t) {
    if (launch_sides(h->cx->args.x[0], h->cx->args.x[1], h->cs->args.x[0], h->cs->args.x[1], h->cx->args.ctrl,
                     h->cs->args.ctrl, h->n, h->p.B, h->p.l, h->dtype, h->stream) != hipSuccess)
      return poison(h, hipErrorLaunchFailure);
    deco_status st = launch_steps(h->cs, 1, 1, 0);
    if (!st) st = launch_steps(h->cx, 1, 1, 0);
    if (st) {
      h->poisoned = true;
      return st;
    }
  }
  return DECO_OK;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// The two parameter sets of a many-component handle (see deco_handle::cx).
void wide_params(const deco_params* p, deco_params* px, deco_params* ps) {
  *px = *p;
  px->B = p->l * p->B;
  px->l = 1;
  px->lifted = 0;
  px->score_every = 1 << 30;  // the iterate handle's own (unlifted) rounding is never used
  *ps = *p;
  ps->l = 1;
  ps->lifted = 1;
  ps->eta = 0.0f;
}

size_t wide_sum_bytes(long long n, const deco_params* p) { return align_up((size_t)n * p->B * elem_size(p->x_dtype)); }

hipError_t wide_sides(deco_handle* h, bool into_start_buffer) {
  deco_handle* x = h->cx;
  deco_handle* c = h->cs;
  if (into_start_buffer)
    return launch_sides(x->args.x[x->t_host & 1], x->args.x[x->t_host & 1], h->sbuf, h->sbuf, nullptr, nullptr, h->n,
                        h->p.B, h->p.l, h->dtype, h->stream);
  return launch_sides(x->args.x[0], x->args.x[1], c->args.x[0], c->args.x[1], x->args.ctrl, c->args.ctrl, h->n,
                      h->p.B, h->p.l, h->dtype, h->stream);
}

deco_status wide_poison(deco_handle* h, deco_status st) {
  if (st == DECO_E_DEVICE || st == DECO_E_STATE) h->poisoned = true;
  return st;
}

}  // namespace

extern "C" {

const char* deco_status_string(deco_status s) {
  switch (s) {
    case DECO_OK: return "ok";
    case DECO_E_INVAL: return "invalid argument or graph";
    case DECO_E_NOMEM: return "workspace too small or allocation failed";
    case DECO_E_DEVICE: return "device error";
    case DECO_E_STATE: return "handle poisoned by an earlier device error";
    case DECO_E_NONFINITE: return "non-finite weight or starting value";
    case DECO_E_UNSUPPORTED: return "unsupported shape";
    default: return "unknown status";
  }
}

deco_status deco_workspace_size(const deco_graph* g, const deco_params* p, size_t* bytes) {
  deco_status st = check_graph_args(g);
  if (st) return st;
  if ((st = check_params(p))) return st;
  if (!bytes) return DECO_E_INVAL;
  if (p->l > kMaxL) {
    deco_params px, ps;
    wide_params(p, &px, &ps);
    *bytes = align_up(layout_for(g->n, g->nnz, g->num_graphs, &px, g->w != nullptr).total) +
             align_up(layout_for(g->n, g->nnz, g->num_graphs, &ps, g->w != nullptr).total) +
             2 * wide_sum_bytes(g->n, p);
    return DECO_OK;
  }
  *bytes = layout_for(g->n, g->nnz, g->num_graphs, p, g->w != nullptr).total;
  return DECO_OK;
}

deco_status deco_init(deco_handle** out, const deco_graph* g, const deco_params* p, void* X,
                      void* workspace, size_t workspace_bytes, void* stream) {
  if (!out) return DECO_E_INVAL;
  *out = nullptr;
  deco_status st = check_graph_args(g);
  if (st) return st;
  if ((st = check_params(p))) return st;
  if (!X || !workspace) return DECO_E_INVAL;
  if (((uintptr_t)X % 16) != 0 || ((uintptr_t)workspace % kAlign) != 0) return DECO_E_INVAL;
  if (p->l > kMaxL) {
    size_t need = 0;
    if ((st = deco_workspace_size(g, p, &need))) return st;
    if (workspace_bytes < need) return DECO_E_NOMEM;
    deco_params px, ps;
    wide_params(p, &px, &ps);
    const size_t wx = align_up(layout_for(g->n, g->nnz, g->num_graphs, &px, g->w != nullptr).total);
    const size_t wsz = align_up(layout_for(g->n, g->nnz, g->num_graphs, &ps, g->w != nullptr).total);
    char* base = reinterpret_cast<char*>(workspace);
    char* xs = base + wx + wsz;  // the score handle's iterate (n x B)
    deco_handle* h = new deco_handle();
    h->g = *g;
    h->p = *p;
    h->stream = reinterpret_cast<hipStream_t>(stream);
    h->n = g->n;
    h->nnz = g->nnz;
    h->G = g->num_graphs;
    h->C = p->l * p->B;
    h->NBY = nby_of(p->B);
    h->dtype = p->x_dtype;
    h->unit = g->w == nullptr;
    h->X = X;
    h->sbuf = xs + wide_sum_bytes(g->n, p);
    if ((st = deco_init(&h->cx, g, &px, X, base, wx, stream)) || (st = deco_init(&h->cs, g, &ps, xs, base + wx, wsz,
                                                                                  stream))) {
      deco_destroy(h);
      return st;
    }
    h->R = h->cs->R;
    *out = h;
    return DECO_OK;
  }
  Layout lay = layout_for(g->n, g->nnz, g->num_graphs, p, g->w != nullptr);
  if (workspace_bytes < lay.total) return DECO_E_NOMEM;

  deco_handle* h = new deco_handle();
  h->g = *g;
  h->p = *p;
  h->stream = reinterpret_cast<hipStream_t>(stream);
  h->n = g->n;
  h->nnz = g->nnz;
  h->G = g->num_graphs;
  h->C = p->l * p->B;
  h->NBY = nby_of(p->B);
  h->R = lay.R;
  h->dtype = p->x_dtype;
  h->unit = g->w == nullptr;
  h->lay = lay;
  h->ws = reinterpret_cast<char*>(workspace);
  h->X = X;

  // host copies of the row structure (schedule, IDI statistics, DUI maxima)
  h->rp_host.resize(g->n + 1);
  hipError_t e = hipMemcpyAsync(h->rp_host.data(), g->row_ptr, sizeof(int) * (g->n + 1),
                                hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    delete h;
    return DECO_E_DEVICE;
  }
  h->goff_host.assign(h->G + 1, 0);
  if (g->graph_row_offset) {
    e = hipMemcpyAsync(h->goff_host.data(), g->graph_row_offset, sizeof(int) * (h->G + 1),
                       hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
      delete h;
      return DECO_E_DEVICE;
    }
  } else {
    h->goff_host[1] = (int)g->n;
  }
  bool ok = h->rp_host[0] == 0 && h->rp_host[g->n] == g->nnz;
  for (long long v = 0; ok && v < g->n; ++v) ok = h->rp_host[v] <= h->rp_host[v + 1];
  ok = ok && h->goff_host[0] == 0 && h->goff_host[h->G] == g->n;
  for (int i = 0; ok && i < h->G; ++i) ok = h->goff_host[i] < h->goff_host[i + 1];
  if (!ok) {
    delete h;
    return DECO_E_INVAL;
  }
  char* ws = h->ws;
  StepArgs& a = h->args;
  a.rp = g->row_ptr;
  a.ci = g->col_idx;
  a.w = g->w;
  a.dw = reinterpret_cast<float*>(ws + lay.dw);
  a.x[0] = X;
  a.x[1] = ws + lay.xalt;
  a.C = h->C;
  a.B = p->B;
  a.L = p->l;
  a.lifted = p->lifted;
  a.slots = reinterpret_cast<int*>(ws + lay.slots);
  a.sw = g->w ? reinterpret_cast<float*>(ws + lay.sw) : nullptr;
  a.items = reinterpret_cast<int4*>(ws + lay.items);
  a.seg = reinterpret_cast<int*>(ws + lay.seg);
  a.cW = p->grad_form == DECO_GRAD_CUT ? -0.5f : -1.0f;
  a.cD = p->grad_form == DECO_GRAD_CUT ? 0.0f : 1.0f;
  a.eta = reinterpret_cast<float*>(ws + lay.eta);
  a.bits[0] = reinterpret_cast<uint8_t*>(ws + lay.bits0);
  a.bits[1] = reinterpret_cast<uint8_t*>(ws + lay.bits1);
  a.bits[2] = reinterpret_cast<uint8_t*>(ws + lay.bits2);
  a.best_bits = reinterpret_cast<uint8_t*>(ws + lay.best_bits);
  a.mask = reinterpret_cast<uint8_t*>(ws + lay.mask);
  a.NBY = h->NBY;
  a.acc = reinterpret_cast<double*>(ws + lay.acc);
  a.R = lay.R;
  a.G = h->G;
  a.nextra = completion_blocks((long long)h->G * p->B);
  a.cur_cut = reinterpret_cast<double*>(ws + lay.cur_cut);
  a.best_cut = reinterpret_cast<double*>(ws + lay.best_cut);
  a.best_step = reinterpret_cast<int*>(ws + lay.best_step);
  a.trace = nullptr;
  a.trace_cap = 1;
  a.ctrl = reinterpret_cast<DevCtrl*>(ws + lay.ctrl);
  a.do_update = 1;
  a.cut_scale = 0.5;
  a.dense_w = nullptr;
  a.n = g->n;

  int* goff_dev = reinterpret_cast<int*>(ws + lay.goff);
  int* flags = reinterpret_cast<int*>(ws + lay.flags);
  int hflags = 0;
  e = hipMemcpyAsync(goff_dev, h->goff_host.data(), sizeof(int) * (h->G + 1), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(flags, 0, sizeof(int) * 4, h->stream);
  if (e == hipSuccess)
    e = launch_validate(g->n, g->row_ptr, g->col_idx, g->w, goff_dev, h->G, const_cast<float*>(a.dw), flags,
                        h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    delete h;
    return DECO_E_DEVICE;
  }
  if (hflags & (1 | 2 | 8)) {
    delete h;
    return DECO_E_INVAL;
  }
  if (hflags & 4) {
    delete h;
    return DECO_E_NONFINITE;
  }
  a.intw = (hflags & 16) ? 0 : 1;
  a.pm1 = (g->w != nullptr && !(hflags & 32)) ? 1 : 0;
  e = launch_build_slots(g->n, g->nnz, g->row_ptr, g->col_idx, g->w, a.dw, const_cast<int*>(a.slots),
                         const_cast<float*>(a.sw), h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    delete h;
    return DECO_E_DEVICE;
  }

  // schedule: cached winner of an earlier autotune for this shape, else the default
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find(cache_key(h));
    h->sched = it != g_cache.end() ? it->second : default_schedule(h);
  }
  if (!build_schedule(h, h->sched)) {
    h->sched = default_schedule(h);
    if (!build_schedule(h, h->sched)) {
      delete h;
      return DECO_E_UNSUPPORTED;
    }
  }
  if (upload_schedule(h) != DECO_OK) {
    delete h;
    return DECO_E_DEVICE;
  }
  e = launch_fill_eta(const_cast<float*>(a.eta), p->B, p->eta, h->stream);
  // every component active until a start says otherwise
  h->lact_host.assign(p->B, p->l);
  a.lact = reinterpret_cast<const int*>(ws + lay.l_active);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + lay.l_active, h->lact_host.data(), sizeof(int) * p->B, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = launch_reset(a, a.acc, 2LL * lay.R * h->G * p->B, p->score_every, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    delete h;
    return DECO_E_DEVICE;
  }
  *out = h;
  return DECO_OK;
}

deco_status deco_start(deco_handle* h, const deco_start_args* s) {
  if (!h || !s) return DECO_E_INVAL;
  if (h->cx) {
    if (h->poisoned) return DECO_E_STATE;
    // iterates: the same start over the l B columns (the draws are per column); active
    // components become per-column 0/1 counts
    deco_start_args a = *s;
    std::vector<int32_t> lc;
    if (s->l_active) {
      lc.resize((size_t)h->C);
      for (int b = 0; b < h->p.B; ++b) {
        if (s->l_active[b] < 0 || s->l_active[b] > h->p.l) return DECO_E_INVAL;
        for (int i = 0; i < h->p.l; ++i) lc[(size_t)i * h->p.B + b] = i < s->l_active[b] ? 1 : 0;
      }
      a.l_active = lc.data();
    }
    deco_status st = deco_start(h->cx, &a);
    if (st) return wide_poison(h, st);
    // scores: the component sums of the start
    if (wide_sides(h, true) != hipSuccess) return wide_poison(h, DECO_E_DEVICE);
    deco_start_args b{};
    b.kind = DECO_INIT_USER;
    b.x0 = h->sbuf;
    b.scale = 1.0;
    if ((st = deco_start(h->cs, &b))) return wide_poison(h, st);
    h->t_host = 0;
    for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
    return DECO_OK;
  }
  if (h->poisoned) return DECO_E_STATE;
  if (s->kind < DECO_INIT_USER || s->kind > DECO_INIT_LEARNED) return DECO_E_INVAL;
  if (s->kind == DECO_INIT_LEARNED && !s->magnitude) return DECO_E_INVAL;
  if (s->kind == DECO_INIT_USER && !s->x0) return DECO_E_INVAL;
  if (s->kind == DECO_INIT_MEAN && !s->mean_z) return DECO_E_INVAL;
  if (h->dense && (s->kind == DECO_INIT_DUI || s->kind == DECO_INIT_IDI || s->kind == DECO_INIT_LEARNED))
    return DECO_E_UNSUPPORTED;
  if (!(s->scale > 0.0) || !(s->sigma2 >= 0.0) || !std::isfinite(s->scale) || !std::isfinite(s->sigma2))
    return DECO_E_INVAL;
  char* ws = h->ws;
  const Layout& lay = h->lay;
  int* lact = nullptr;
  if (s->l_active) {
    for (int b = 0; b < h->p.B; ++b)
      if (s->l_active[b] < 0 || s->l_active[b] > h->p.l) return DECO_E_INVAL;
  }
  if (!h->dense) {
    // the step kernel gathers only the active components (the start zeroes the others)
    bool same = true;
    for (int b = 0; b < h->p.B; ++b) same = same && h->lact_host[b] == (s->l_active ? s->l_active[b] : h->p.l);
    if (!same) {
      for (int b = 0; b < h->p.B; ++b) h->lact_host[b] = s->l_active ? s->l_active[b] : h->p.l;
      HIP_TRY(h, hipMemcpyAsync(ws + lay.l_active, h->lact_host.data(), sizeof(int) * h->p.B, hipMemcpyHostToDevice,
                                h->stream));
    }
    if (s->l_active) lact = reinterpret_cast<int*>(ws + lay.l_active);
    // the step kernel runs the largest active count of components (at least 1)
    int lrun = 1;
    for (int b = 0; b < h->p.B; ++b) lrun = std::max(lrun, h->lact_host[b]);
    if (lrun != h->args.L) {
      // captured launches hold another step kernel
      h->args.L = lrun;
      for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
      h->graphs.clear();
    }
  }
  int* goff_dev = reinterpret_cast<int*>(ws + lay.goff);
  if (s->kind == DECO_INIT_USER) {
    int* flags = reinterpret_cast<int*>(ws + lay.flags) + 1;
    int nf = 0;
    HIP_TRY(h, hipMemsetAsync(flags, 0, sizeof(int), h->stream));
    HIP_TRY(h, launch_convert_user(s->x0, h->X, h->n * h->C, h->dtype, lact, h->C, h->p.B, flags, h->stream));
    HIP_TRY(h, hipMemcpyAsync(&nf, flags, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (nf) return DECO_E_NONFINITE;
  } else {
    InitArgs ia{};
    ia.n = h->n;
    ia.C = h->C;
    ia.B = h->p.B;
    ia.L = h->p.l;
    ia.rp = h->g.row_ptr;
    ia.ci = h->g.col_idx;
    ia.w = h->g.w;
    ia.goff = goff_dev;
    ia.G = h->G;
    ia.mean_z = s->mean_z;
    ia.l_active = lact;
    ia.scratch = reinterpret_cast<int8_t*>(ws + lay.xalt);
    ia.scale = s->scale;
    ia.sd = std::sqrt(s->sigma2);
    ia.seed = h->p.seed;
    ia.batch = s->batch;
    ia.kind = s->kind;
    ia.dtype = h->dtype;
    ia.X = h->X;
    double* thr = reinterpret_cast<double*>(ws + lay.thr);
    int* delta = reinterpret_cast<int*>(ws + lay.delta);
    ia.magnitude = s->magnitude;
    if (s->kind == DECO_INIT_IDI || s->kind == DECO_INIT_DUI || s->kind == DECO_INIT_LEARNED) {
      // per-graph degree statistics on the host copy of row_ptr (Sec. 4.1)
      std::vector<double> th(h->G);
      std::vector<int> dl(h->G);
      for (int gi = 0; gi < h->G; ++gi) {
        const int r0 = h->goff_host[gi], r1 = h->goff_host[gi + 1];
        const double cnt = (double)(r1 - r0);
        double sum = 0.0;
        int mx = 0;
        for (int v = r0; v < r1; ++v) {
          const int d = h->rp_host[v + 1] - h->rp_host[v];
          sum += (double)d;
          mx = std::max(mx, d);
        }
        const double mean = sum / cnt;
        double ss = 0.0;
        for (int v = r0; v < r1; ++v) {
          const double dev = (double)(h->rp_host[v + 1] - h->rp_host[v]) - mean;
          ss += dev * dev;
        }
        th[gi] = mean + s->beta * std::sqrt(ss / cnt);
        dl[gi] = mx;
      }
      HIP_TRY(h, hipMemcpyAsync(thr, th.data(), sizeof(double) * h->G, hipMemcpyHostToDevice, h->stream));
      HIP_TRY(h, hipMemcpyAsync(delta, dl.data(), sizeof(int) * h->G, hipMemcpyHostToDevice, h->stream));
      HIP_TRY(h, hipStreamSynchronize(h->stream));
    }
    ia.thr = thr;
    ia.delta = delta;
    HIP_TRY(h, launch_init(ia, h->stream));
  }
  if (h->dense) HIP_TRY(h, launch_dense_transpose(h->X, h->args.xT[0], h->n, h->C, h->stream));
  // components past the step kernel's count are never written by the steps: the start wrote
  // them as 0 into X_0; the other buffer (the start's scratch, and earlier batches may have run
  // more components) is cleared
  if (!h->dense && h->args.L < h->p.l)
    HIP_TRY(h, launch_zero(ws + lay.xalt, (size_t)h->n * h->C * elem_size(h->dtype), h->stream));
  if (h->args.vel)  // a new start begins at rest
    HIP_TRY(h, hipMemsetAsync(h->args.vel, 0, sizeof(float) * (size_t)h->n * h->C, h->stream));
  HIP_TRY(h, launch_reset(h->args, h->args.acc, 2LL * h->R * h->G * h->p.B, h->p.score_every, h->stream));
  h->t_host = 0;
  return DECO_OK;
}

deco_status deco_set_eta(deco_handle* h, const float* eta_host) {
  if (!h || !eta_host) return DECO_E_INVAL;
  if (h->poisoned) return DECO_E_STATE;
  if (h->cx) {
    std::vector<float> e((size_t)h->C);
    for (int i = 0; i < h->p.l; ++i)
      for (int b = 0; b < h->p.B; ++b) e[(size_t)i * h->p.B + b] = eta_host[b];
    return wide_poison(h, deco_set_eta(h->cx, e.data()));
  }
  for (int b = 0; b < h->p.B; ++b)
    if (!std::isfinite(eta_host[b])) return DECO_E_NONFINITE;
  HIP_TRY(h, hipMemcpyAsync(const_cast<float*>(h->args.eta), eta_host, sizeof(float) * h->p.B,
                            hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return DECO_OK;
}

deco_status deco_set_momentum(deco_handle* h, float mu, float* velocity) {
  if (!h) return DECO_E_INVAL;
  if (h->poisoned) return DECO_E_STATE;
  if (h->cx) {
    for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
    return wide_poison(h, deco_set_momentum(h->cx, mu, velocity));
  }
  if (h->dense) return DECO_E_UNSUPPORTED;
  if (!std::isfinite(mu)) return DECO_E_NONFINITE;
  h->args.vel = velocity;
  h->args.mu = velocity ? mu : 0.0f;
  // captured step graphs hold the old arguments
  for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
  h->graphs.clear();
  if (velocity)
    HIP_TRY(h, hipMemsetAsync(velocity, 0, sizeof(float) * (size_t)h->n * h->C, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return DECO_OK;
}

deco_status deco_step(deco_handle* h, int32_t steps, int32_t use_graph) {
  if (!h || steps < 0) return DECO_E_INVAL;
  if (h->poisoned) return DECO_E_STATE;
  if (steps == 0) return DECO_OK;
  if (!use_graph) {
    deco_status st = h->cx ? wide_launch_steps(h, steps) : launch_steps(h, steps, 1, 0);
    if (st) return st;
  } else {
    if (h->stream == nullptr) return DECO_E_INVAL;
    auto it = h->graphs.find(steps);
    if (it == h->graphs.end()) {
      hipGraph_t graph;
      HIP_TRY(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
      deco_status st = h->cx ? wide_launch_steps(h, steps) : launch_steps(h, steps, 1, 0);
      hipError_t e = hipStreamEndCapture(h->stream, &graph);
      if (st) return st;
      HIP_TRY(h, e);
      hipGraphExec_t exec;
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      HIP_TRY(h, e);
      it = h->graphs.emplace(steps, exec).first;
    }
    HIP_TRY(h, hipGraphLaunch(it->second, h->stream));
  }
  h->t_host += steps;
  if (h->cx) {
    for (deco_handle* c : {h->cx, h->cs}) {
      c->t_host += steps;
      HIP_TRY(h, launch_drain(c->args, c->n, reinterpret_cast<int*>(c->ws + c->lay.goff), c->stream));
    }
    return DECO_OK;
  }
  HIP_TRY(h, launch_drain(h->args, h->n, reinterpret_cast<int*>(h->ws + h->lay.goff), h->stream));
  return DECO_OK;
}

deco_status deco_round_score(deco_handle* h, double* cut_out, uint8_t* bits_out) {
  if (!h) return DECO_E_INVAL;
  if (h->poisoned) return DECO_E_STATE;
  if (h->cx) {
    if (wide_sides(h, false) != hipSuccess) return wide_poison(h, DECO_E_DEVICE);
    return wide_poison(h, deco_round_score(h->cs, cut_out, bits_out));
  }
  deco_status st = launch_steps(h, 1, 0, 1);
  if (st) return st;
  HIP_TRY(h, launch_drain(h->args, h->n, reinterpret_cast<int*>(h->ws + h->lay.goff), h->stream));
  const size_t gb = (size_t)h->G * h->p.B;
  if (cut_out)
    HIP_TRY(h, hipMemcpyAsync(cut_out, h->args.cur_cut, sizeof(double) * gb, hipMemcpyDeviceToDevice, h->stream));
  if (bits_out)
    HIP_TRY(h, hipMemcpyAsync(bits_out, h->args.bits[h->t_host % 3], (size_t)h->n * h->NBY,
                              hipMemcpyDeviceToDevice, h->stream));
  return DECO_OK;
}

deco_status deco_best(deco_handle* h, double* best_cut, int32_t* best_step, uint8_t* best_bits) {
  if (!h || !best_cut) return DECO_E_INVAL;
  if (h->poisoned) return DECO_E_STATE;
  if (h->cx) return wide_poison(h, deco_best(h->cs, best_cut, best_step, best_bits));
  const size_t gb = (size_t)h->G * h->p.B;
  const int* goff_dev = reinterpret_cast<int*>(h->ws + h->lay.goff);
  HIP_TRY(h, launch_drain(h->args, h->n, goff_dev, h->stream));
  HIP_TRY(h, hipMemcpyAsync(best_cut, h->args.best_cut, sizeof(double) * gb, hipMemcpyDeviceToHost, h->stream));
  if (best_step)
    HIP_TRY(h, hipMemcpyAsync(best_step, h->args.best_step, sizeof(int) * gb, hipMemcpyDeviceToHost, h->stream));
  if (best_bits)
    HIP_TRY(h, hipMemcpyAsync(best_bits, h->args.best_bits, (size_t)h->n * h->NBY, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return DECO_OK;
}

deco_status deco_read_x(deco_handle* h, void* dst) {
  if (!h || !dst) return DECO_E_INVAL;
  if (h->poisoned) return DECO_E_STATE;
  if (h->cx) return wide_poison(h, deco_read_x(h->cx, dst));
  HIP_TRY(h, hipMemcpyAsync(dst, h->args.x[h->t_host & 1], (size_t)h->n * h->C * elem_size(h->dtype),
                            hipMemcpyDeviceToDevice, h->stream));
  return DECO_OK;
}

deco_status deco_set_trace(deco_handle* h, double* trace, int32_t capacity) {
  if (!h || (trace && capacity < 1)) return DECO_E_INVAL;
  if (h->cx) {
    deco_status st = deco_set_trace(h->cs, trace, capacity);
    if (st) return st;
  }
  h->args.trace = trace;
  h->args.trace_cap = trace ? capacity : 1;
  for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
  h->graphs.clear();
  return DECO_OK;
}

int64_t deco_current_step(const deco_handle* h) { return h ? h->t_host : -1; }

deco_status deco_autotune(deco_handle* h, int32_t steps) {
  if (!h || steps < 1) return DECO_E_INVAL;
  if (h->poisoned) return DECO_E_STATE;
  if (h->cx) {
    deco_status st = deco_autotune(h->cx, steps);
    if (!st) st = deco_autotune(h->cs, steps);
    for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
    return wide_poison(h, st);
  }
  if (h->dense) return DECO_OK;  // one fixed tiling
  const Schedule base = default_schedule(h);
  std::vector<Schedule> cand;
  const int vec = base.vec;
  // tiles of a quarter of the widest and up (narrower lifted tiles, each XCD owning its own,
  // were measured slower at BA(10^4, 4), B = 256: set_schedule still accepts them)
  const int mt = min_tile(h->p.B, h->p.l);
  const int wspan = 4;
  // lane widths: the native one, and 4 values per lane for unlifted bfloat16 rows (twice the
  // lanes per tile: one row team per wave at B = 256) and lifted float32 rows (half the lanes
  // per tile, twice the registers per lane)
  std::vector<int> vecs{vec};
  if ((h->dtype == DECO_BF16 && vec == 8) || (h->dtype == DECO_F32 && vec == 2)) vecs.push_back(4);
  if (h->dtype == DECO_BF16 && vec == 4 && h->p.l >= 2 && h->p.l <= 8) vecs.push_back(2);
  for (int vw : vecs) {
    const int wmax_v = max_wc(vw, h->p.B);
    for (int Wc = wmax_v; Wc >= 1 && Wc * vw >= mt && Wc * wspan >= wmax_v; Wc /= 2) {
      for (int npi : {128, 256, 512, 1024, 2048}) {
        for (int mode = 0; mode < 2; ++mode) {
          if (mode == 1 && h->p.B / (Wc * vw) < 2) continue;
          for (int bpx : {64, 256, kMaxBlocksPerXcd}) {
            Schedule s = base;
            s.vec = vw;
            s.Wc = Wc;
            s.xcd_mode = mode;
            s.blocks_per_xcd = bpx;
            s.nnz_per_item = npi;
            cand.push_back(s);
          }
        }
      }
    }
  }
  // resident schedules (all steps of a call in one launch, each workgroup's tile in LDS) for
  // every tile width that fits
  if (h->p.l == 1)
    for (int bt : {1, 2, 4, 8, 16}) {
      Schedule s = base;
      s.rbt = bt;
      cand.push_back(s);
    }
  hipEvent_t e0, e1;
  HIP_TRY(h, hipEventCreate(&e0));
  HIP_TRY(h, hipEventCreate(&e1));
  // Every candidate is timed twice (the faster run counts), then the four fastest are timed
  // three more times each and the fastest of those runs wins; a near-tie (within 3%) keeps
  // the candidate that came first (the default comes first). Step-kernel candidates cost the
  // same per step at any call length and are timed over at most kStepTrial steps; resident
  // ones carry a fixed cost per call and are timed over the whole call.
  constexpr int kStepTrial = 50, kFinalists = 4;
  cand.insert(cand.begin(), base);
  deco_start_args sa{};
  sa.kind = DECO_INIT_UNIFORM;
  sa.scale = 1.0;
  // time per step (ms) of candidate s, the fastest of 'reps' calls; 1e30 when it does not fit
  auto trial = [&](Schedule& s, int reps, float* out) -> deco_status {
    *out = 1e30f;
    if (!build_schedule(h, s)) return DECO_OK;
    h->sched = s;
    if (upload_schedule(h) != DECO_OK) return DECO_E_DEVICE;
    deco_status st = deco_start(h, &sa);
    if (st) return st;
    if ((st = launch_steps(h, 2, 1, 0))) return st;  // warm caches
    const int n_steps = s.rbt > 0 ? steps : std::min(steps, kStepTrial);
    for (int rep = 0; rep < reps; ++rep) {
      HIP_TRY(h, hipEventRecord(e0, h->stream));
      if ((st = launch_steps(h, n_steps, 1, 0))) return st;
      HIP_TRY(h, hipEventRecord(e1, h->stream));
      HIP_TRY(h, hipEventSynchronize(e1));
      float r = 0.0f;
      HIP_TRY(h, hipEventElapsedTime(&r, e0, e1));
      *out = std::min(*out, r / (float)n_steps);
    }
    return DECO_OK;
  };
  std::vector<std::pair<float, int>> timed;
  for (int i = 0; i < (int)cand.size(); ++i) {
    float ms;
    deco_status st = trial(cand[i], 2, &ms);
    if (st) return st;
    if (ms < 1e30f) timed.emplace_back(ms, i);
  }
  std::sort(timed.begin(), timed.end());
  if (timed.size() > (size_t)kFinalists) timed.resize(kFinalists);
  std::sort(timed.begin(), timed.end(), [](const std::pair<float, int>& x, const std::pair<float, int>& y) {
    return x.second < y.second;
  });
  float best_ms = 1e30f;
  Schedule best = h->sched;
  for (auto& f : timed) {
    float ms;
    deco_status st = trial(cand[f.second], 3, &ms);
    if (st) return st;
    ms = std::min(ms, f.first);
    if (ms < 0.97f * best_ms) {
      best_ms = ms;
      best = cand[f.second];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->sched = best;
  if (!build_schedule(h, h->sched)) return DECO_E_UNSUPPORTED;
  deco_status st = upload_schedule(h);
  if (st) return st;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    Schedule keep = h->sched;
    keep.items.clear();
    keep.ritems.clear();
    keep.rgs.clear();
    g_cache[cache_key(h)] = keep;
  }
  return deco_start(h, &sa);
}

deco_status deco_set_schedule(deco_handle* h, const deco_schedule* q) {
  if (!h || !q) return DECO_E_INVAL;
  if (h->poisoned) return DECO_E_STATE;
  if (h->cx) {  // the iterate handle's schedule (the score handle keeps its own)
    for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
    return wide_poison(h, deco_set_schedule(h->cx, q));
  }
  if (h->dense) return DECO_E_UNSUPPORTED;
  if (q->lanes_per_row < 1 || (q->lanes_per_row & (q->lanes_per_row - 1)) ||
      q->blocks_per_xcd < 1 || q->blocks_per_xcd > kMaxBlocksPerXcd || q->nnz_per_item < kMinItemSlots ||
      q->nnz_per_item > kEmax || q->long_row < 16 ||
      (q->xcd_mode != 0 && q->xcd_mode != 1))
    return DECO_E_INVAL;
  Schedule s = default_schedule(h);
  if (q->lane_elems != 0) {
    // the alternative widths: 4 values per lane (unlifted bfloat16 rows, float32 rows of 2 to
    // 8 components) and 2 (bfloat16 rows of 2 to 8 components)
    if (q->lane_elems == 2 && h->dtype == DECO_BF16 && s.vec == 4 && h->p.l >= 2 && h->p.l <= 8) {
      s.vec = 2;
    } else {
      if (q->lane_elems != 4 || !((h->dtype == DECO_BF16 && s.vec == 8) || (h->dtype == DECO_F32 && s.vec == 2)))
        return DECO_E_INVAL;
      s.vec = 4;
    }
  }
  s.Wc = q->lanes_per_row;
  s.dlong = q->long_row;
  s.xcd_mode = q->xcd_mode;
  s.blocks_per_xcd = q->blocks_per_xcd;
  s.nnz_per_item = q->nnz_per_item;
  if (q->resident_cols < 0) return DECO_E_INVAL;
  if (q->resident_cols > 0) {
    s = default_schedule(h);  // the step kernel's part (score-only passes, momentum) as by default
    s.rbt = q->resident_cols;
  }
  if (!build_schedule(h, s)) return s.rbt > 0 ? DECO_E_UNSUPPORTED : DECO_E_INVAL;
  h->sched = std::move(s);
  return upload_schedule(h);
}

deco_status deco_schedule_string(const deco_handle* h, char* buf, int32_t cap) {
  if (!h || !buf || cap < 1) return DECO_E_INVAL;
  if (h->cx) {
    char a[256], b[256];
    deco_schedule_string(h->cx, a, sizeof(a));
    deco_schedule_string(h->cs, b, sizeof(b));
    std::snprintf(buf, (size_t)cap, "l=%d over %d columns: %s | sums: %s", h->p.l, h->C, a, b);
    return DECO_OK;
  }
  if (h->dense) {
    std::snprintf(buf, (size_t)cap, "dense bf16 MFMA 32x32x16: tiles 128x128x64, grid=%lld, R=%d",
                  (long long)(h->n / 128) * (2 * h->C / 128), h->R);
    return DECO_OK;
  }
  const Schedule& s = h->sched;
  if (s.rbt > 0) {
    std::snprintf(buf, (size_t)cap, "resident cols=%d items=%d max_rows=%d lds=%zu | vec=%d Wc=%d R=%d", s.rbt,
                  (int)s.ritems.size(), s.rmax_rows, resident_lds_bytes(s.rmax_rows, s.rbt, h->dtype), s.vec, s.Wc,
                  h->R);
    return DECO_OK;
  }
  std::snprintf(buf, (size_t)cap,
                "vec=%d Wc=%d dlong=%d tile=%d tiles=%d xcd_mode=%d grid=%d items=%d "
                "rows_per_item=%d nnz_per_item=%d R=%d",
                s.vec, s.Wc, s.dlong, s.Wc * s.vec, h->p.B / (s.Wc * s.vec), s.xcd_mode, s.grid, s.nitems,
                s.rows_per_item, s.nnz_per_item, h->R);
  return DECO_OK;
}


deco_status deco_dense_workspace_size(int64_t n, const deco_params* p, size_t* bytes) {
  deco_status st = check_params(p);
  if (st) return st;
  if (!bytes || n < 1) return DECO_E_INVAL;
  if (n % 128 != 0 || p->B % 128 != 0 || p->l != 1 || p->lifted || p->x_dtype != DECO_BF16 || n >= (1LL << 31))
    return DECO_E_UNSUPPORTED;
  *bytes = layout_for(n, 0, 1, p, false, true).total;
  return DECO_OK;
}

deco_status deco_dense_init(deco_handle** out, int64_t n, const void* W, const deco_params* p, void* X,
                            void* workspace, size_t workspace_bytes, void* stream) {
  if (!out) return DECO_E_INVAL;
  *out = nullptr;
  size_t need = 0;
  deco_status st = deco_dense_workspace_size(n, p, &need);
  if (st) return st;
  if (!W || !X || !workspace) return DECO_E_INVAL;
  if (((uintptr_t)X % 16) != 0 || ((uintptr_t)W % 16) != 0 || ((uintptr_t)workspace % kAlign) != 0)
    return DECO_E_INVAL;
  if (workspace_bytes < need) return DECO_E_NOMEM;
  const Layout lay = layout_for(n, 0, 1, p, false, true);
  deco_handle* h = new deco_handle();
  h->dense = true;
  h->p = *p;
  h->g.n = n;
  h->g.nnz = 0;
  h->g.num_graphs = 1;
  h->stream = reinterpret_cast<hipStream_t>(stream);
  h->n = n;
  h->G = 1;
  h->C = p->B;
  h->NBY = nby_of(p->B);
  h->R = lay.R;
  h->dtype = DECO_BF16;
  h->unit = false;
  h->lay = lay;
  h->ws = reinterpret_cast<char*>(workspace);
  h->X = X;
  h->goff_host = {0, (int)n};
  char* ws = h->ws;
  StepArgs& a = h->args;
  a.dw = reinterpret_cast<float*>(ws + lay.dw);
  a.x[0] = X;
  a.x[1] = ws + lay.xalt;
  a.C = h->C;
  a.B = p->B;
  a.L = 1;
  a.lifted = 0;
  a.cW = p->grad_form == DECO_GRAD_CUT ? -0.5f : -1.0f;
  a.cD = p->grad_form == DECO_GRAD_CUT ? 0.0f : 1.0f;
  a.eta = reinterpret_cast<float*>(ws + lay.eta);
  a.bits[0] = reinterpret_cast<uint8_t*>(ws + lay.bits0);
  a.bits[1] = reinterpret_cast<uint8_t*>(ws + lay.bits1);
  a.bits[2] = reinterpret_cast<uint8_t*>(ws + lay.bits2);
  a.best_bits = reinterpret_cast<uint8_t*>(ws + lay.best_bits);
  a.mask = reinterpret_cast<uint8_t*>(ws + lay.mask);
  a.NBY = h->NBY;
  a.acc = reinterpret_cast<double*>(ws + lay.acc);
  a.R = lay.R;
  a.G = 1;
  a.nextra = 0;
  a.cur_cut = reinterpret_cast<double*>(ws + lay.cur_cut);
  a.best_cut = reinterpret_cast<double*>(ws + lay.best_cut);
  a.best_step = reinterpret_cast<int*>(ws + lay.best_step);
  a.trace = nullptr;
  a.trace_cap = 1;
  a.ctrl = reinterpret_cast<DevCtrl*>(ws + lay.ctrl);
  a.do_update = 1;
  a.cut_scale = 0.25;
  a.dense_w = reinterpret_cast<const uint16_t*>(W);
  a.xT[0] = ws + lay.xt0;
  a.xT[1] = ws + lay.xt1;
  a.n = n;
  int* goff_dev = reinterpret_cast<int*>(ws + lay.goff);
  int* flags = reinterpret_cast<int*>(ws + lay.flags);
  int hflags = 0;
  hipError_t e = hipMemcpyAsync(goff_dev, h->goff_host.data(), sizeof(int) * 2, hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(flags, 0, sizeof(int) * 4, h->stream);
  if (e == hipSuccess) e = launch_dense_validate(a.dense_w, (int)n, const_cast<float*>(a.dw), flags, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&hflags, flags, sizeof(int), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    delete h;
    return DECO_E_DEVICE;
  }
  if (hflags & (1 | 2)) {
    delete h;
    return DECO_E_INVAL;
  }
  if (hflags & 4) {
    delete h;
    return DECO_E_NONFINITE;
  }
  if (hflags & (16 | 32)) {  // the exact score needs integer weights with row sums of |w| <= 2^24
    delete h;
    return DECO_E_UNSUPPORTED;
  }
  a.intw = 1;
  e = launch_fill_eta(const_cast<float*>(a.eta), p->B, p->eta, h->stream);
  if (e == hipSuccess) e = launch_reset(a, a.acc, 2LL * lay.R * p->B, p->score_every, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    delete h;
    return DECO_E_DEVICE;
  }
  *out = h;
  return DECO_OK;
}

void deco_destroy(deco_handle* h) {
  if (!h) return;
  for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
  if (h->cx) deco_destroy(h->cx);
  if (h->cs) deco_destroy(h->cs);
  delete h;
}

void deco_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  philox4x32_10(c, key[0], key[1]);
  for (int i = 0; i < 4; ++i) out[i] = c[i];
}

deco_status deco_philox_device(uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed, int32_t count,
                               uint32_t* out, void* stream) {
  if (count < 0 || (count > 0 && !out)) return DECO_E_INVAL;
  hipError_t e = launch_philox_test(c1, c2, c3, seed, count, out, reinterpret_cast<hipStream_t>(stream));
  return e == hipSuccess ? DECO_OK : DECO_E_DEVICE;
}

static double box_muller(uint32_t r0, uint32_t r1) {
  const double u1 = ((double)(r0 >> 8) + 1.0) * (1.0 / 16777216.0);
  const double u2 = (double)(r1 >> 8) * (1.0 / 16777216.0);
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

deco_status deco_evo_next(int32_t K, const double* fitness, const double* eq, const double* el,
                          const int32_t* l, double lo, double hi, int32_t lmax, uint64_t seed,
                          uint32_t round, double* eq_out, double* el_out, int32_t* l_out) {
  if (K < 1 || !fitness || !eq || !el || !l || !eq_out || !el_out || !l_out || lmax < 1 || !(lo <= hi))
    return DECO_E_INVAL;
  std::vector<int> order(K);
  for (int i = 0; i < K; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return fitness[a] > fitness[b]; });
  const int keep = K / 2;
  std::vector<double> q(K), m(K);
  std::vector<int32_t> ll(K);
  for (int i = 0; i < keep; ++i) {
    q[i] = eq[order[i]];
    m[i] = el[order[i]];
    ll[i] = l[order[i]];
  }
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int i = keep; i < K; ++i) {
    const int src = order[i - keep];
    uint32_t c[4] = {round, (uint32_t)i, kSearch, 0u};
    philox4x32_10(c, k0, k1);
    const double a = eq[src] + 0.2 * box_muller(c[0], c[1]);
    const double b = el[src] + 0.2 * box_muller(c[2], c[3]);
    q[i] = std::min(hi, std::max(lo, a));
    m[i] = std::min(hi, std::max(lo, b));
    uint32_t d[4] = {round, (uint32_t)i, kSearch, 1u};
    philox4x32_10(d, k0, k1);
    const int nl = l[src] + (int)(d[0] % 3u) - 1;
    ll[i] = std::min(lmax, std::max(1, nl));
  }
  for (int i = 0; i < K; ++i) {
    eq_out[i] = q[i];
    el_out[i] = m[i];
    l_out[i] = ll[i];
  }
  return DECO_OK;
}

deco_status deco_evo_init(int32_t K, double lo, double hi, int32_t lmax, int32_t Tq_lo, int32_t Tq_hi, int32_t Tl_lo,
                          int32_t Tl_hi, uint64_t seed, double* eq, double* el, int32_t* l, int32_t* Tq, int32_t* Tl) {
  if (K < 1 || lmax < 1 || !(lo <= hi) || !std::isfinite(lo) || !std::isfinite(hi) || Tq_lo > Tq_hi ||
      Tl_lo > Tl_hi || !eq || !el || !l || !Tq || !Tl)
    return DECO_E_INVAL;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int k = 0; k < K; ++k) {
    uint32_t c[4] = {0xFFFFFFFFu, (uint32_t)k, kSearch, 6u};
    philox4x32_10(c, k0, k1);
    eq[k] = lo + (hi - lo) * ((double)(c[0] >> 8) * (1.0 / 16777216.0));
    el[k] = lo + (hi - lo) * ((double)(c[1] >> 8) * (1.0 / 16777216.0));
    l[k] = 1 + (int32_t)(c[2] % (uint32_t)lmax);
    uint32_t d[4] = {0xFFFFFFFFu, (uint32_t)k, kSearch, 3u};
    philox4x32_10(d, k0, k1);
    Tq[k] = Tq_lo + (int32_t)(d[0] % (uint32_t)((int64_t)Tq_hi - Tq_lo + 1));
    uint32_t e[4] = {0xFFFFFFFFu, (uint32_t)k, kSearch, 5u};
    philox4x32_10(e, k0, k1);
    Tl[k] = Tl_lo + (int32_t)(e[0] % (uint32_t)((int64_t)Tl_hi - Tl_lo + 1));
  }
  return DECO_OK;
}

deco_status deco_evo_next_steps(int32_t K, const double* fitness, const int32_t* T, int32_t T_lo, int32_t T_hi,
                                uint64_t seed, uint32_t round, uint32_t gene, int32_t* T_out) {
  if (K < 1 || !fitness || !T || !T_out || T_lo < 1 || T_lo > T_hi || gene > 1) return DECO_E_INVAL;
  std::vector<int> order(K);
  for (int i = 0; i < K; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return fitness[a] > fitness[b]; });
  const int keep = K / 2;
  std::vector<int32_t> out(K);
  for (int i = 0; i < keep; ++i) out[i] = T[order[i]];
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int i = keep; i < K; ++i) {
    uint32_t c[4] = {round, (uint32_t)i, kSearch, 2u + 2u * gene};
    philox4x32_10(c, k0, k1);
    const double eps = (double)(c[0] >> 8) * (1.0 / 16777216.0);  // eps' ~ U(0, 1)
    const double t = std::floor((double)T[order[i - keep]] * (1.0 + 0.2 * (2.0 * eps - 1.0)));
    out[i] = (int32_t)std::min<double>(T_hi, std::max<double>(T_lo, t));
  }
  for (int i = 0; i < K; ++i) T_out[i] = out[i];
  return DECO_OK;
}

}  // extern "C"

struct deco_solver {
  deco_graph g{};
  deco_solve_params p{};
  hipStream_t s = nullptr;
  char* mem = nullptr;
  deco_handle* hq = nullptr;
  deco_handle* hl = nullptr;
  uint8_t* mean_dev = nullptr;
  int B = 0, K = 0, per = 0, G = 1, lmax = 1, NBY = 1;
  long long n = 0;
  std::vector<double> eq, el, gbest, fit, fitg, bc, target;
  std::vector<int32_t> lk, lact;
  std::vector<int32_t> tq;  // unlifted steps per member (searched when p.T_min > 0)
  std::vector<int32_t> tl;  // lifted steps per member (searched when p.T_l_min > 0)
  std::vector<uint8_t> best_z, zmean, bits;
  std::vector<float> eta;
  std::vector<int> goff;
  int round = 0;
  uint32_t batch = 0;
  long long steps_done = 0;
  double eu = 0.0;
};

namespace {

void solver_free(deco_solver* v) {
  if (!v) return;
  if (v->hq) deco_destroy(v->hq);
  if (v->hl) deco_destroy(v->hl);
  if (v->mem) {
    (void)hipStreamSynchronize(v->s);
    (void)hipFree(v->mem);
  }
  delete v;
}

// Run one batch in which member k steps T[k] times: the batch runs in segments ending at the
// distinct counts, and a member whose count is reached keeps its columns still with a step of
// 0 (the projection leaves an iterate inside the box unchanged). eta holds the members' steps
// and is zeroed in place as they finish. Returns the longest count through *tmax.
// With targets and check_every > 0, the batch also pauses every check_every steps and ends as
// soon as every graph's best (this batch's or an earlier one's) reaches its target (*hit).
deco_status run_counts(deco_solver* v, deco_handle* h, std::vector<float>& eta, const std::vector<int32_t>& T,
                       int* tmax, bool* hit) {
  std::vector<int32_t> ends(T);
  std::sort(ends.begin(), ends.end());
  ends.erase(std::unique(ends.begin(), ends.end()), ends.end());
  const int last = ends.empty() ? 0 : ends.back();
  const bool check = v->p.check_every > 0 && !v->target.empty();
  std::vector<int32_t> stops(ends);
  if (check)
    for (int c = v->p.check_every; c < last; c += v->p.check_every) stops.push_back(c);
  std::sort(stops.begin(), stops.end());
  stops.erase(std::unique(stops.begin(), stops.end()), stops.end());
  deco_status st;
  int done = 0;
  *hit = false;
  for (int32_t e : stops) {
    if (e > done && (st = deco_step(h, e - done, v->p.use_graph))) return st;
    done = std::max(done, (int)e);
    if (e == last) break;
    if (check) {
      if ((st = deco_best(h, v->bc.data(), nullptr, nullptr))) return st;
      bool all = true;
      for (int gi = 0; gi < v->G && all; ++gi) {
        double best = v->gbest[gi];
        for (int b = 0; b < v->B; ++b) best = std::max(best, v->bc[(size_t)gi * v->B + b]);
        all = best >= v->target[gi];
      }
      if (all) {
        *hit = true;
        break;
      }
    }
    bool changed = false;
    for (int b = 0; b < v->B; ++b)
      if (T[b / v->per] == e && eta[b] != 0.0f) {
        eta[b] = 0.0f;
        changed = true;
      }
    if (changed && (st = deco_set_eta(h, eta.data()))) return st;
  }
  *tmax = done;
  return DECO_OK;
}

// Fold one batch's best into the global best, update member fitness (max over the
// member's columns, per graph), and make the batch's best vector the next mean (Sec. 4.2).
deco_status absorb(deco_solver* v, deco_handle* h) {
  deco_status r = deco_best(h, v->bc.data(), nullptr, v->bits.data());
  if (r) return r;
  const int B = v->B, K = v->K, G = v->G;
  for (int gi = 0; gi < G; ++gi) {
    int arg = 0;
    for (int b = 1; b < B; ++b)
      if (v->bc[(size_t)gi * B + b] > v->bc[(size_t)gi * B + arg]) arg = b;
    const double best = v->bc[(size_t)gi * B + arg];
    const bool better = best > v->gbest[gi];
    for (int row = v->goff[gi]; row < v->goff[gi + 1]; ++row) {
      const uint8_t z = (v->bits[(size_t)row * v->NBY + arg / 8] >> (arg % 8)) & 1;
      v->zmean[row] = z;
      if (better) v->best_z[row] = z;
    }
    if (better) v->gbest[gi] = best;
    for (int k = 0; k < K; ++k)
      for (int b = k * v->per; b < (k + 1) * v->per; ++b)
        v->fitg[(size_t)k * G + gi] = std::max(v->fitg[(size_t)k * G + gi], v->bc[(size_t)gi * B + b]);
  }
  if (hipMemcpyAsync(v->mean_dev, v->zmean.data(), (size_t)v->n, hipMemcpyHostToDevice, v->s) != hipSuccess)
    return DECO_E_DEVICE;
  return DECO_OK;
}

}  // namespace

extern "C" {

deco_status deco_solver_create(deco_solver** out, const deco_graph* g, const deco_solve_params* sp, void* stream) {
  if (!out) return DECO_E_INVAL;
  *out = nullptr;
  deco_status st = check_graph_args(g);
  if (st) return st;
  if (!sp) return DECO_E_INVAL;
  if (sp->K < 1 || sp->B < 1 || sp->B % sp->K != 0 || sp->l_max < 1 || sp->T_q < 0 ||
      sp->T_l < 0 || sp->evo_rounds < 0 || !(sp->scale > 0.0) || !(sp->sigma2 >= 0.0) || sp->T_min < 0 ||
      (sp->T_min > 0 && sp->T_min > sp->T_q) || sp->T_l_min < 0 || (sp->T_l_min > 0 && sp->T_l_min > sp->T_l) ||
      sp->check_every < 0 || sp->mode < DECO_SOLVE_DECO || sp->mode > DECO_SOLVE_LIFTED)
    return DECO_E_INVAL;
  if (sp->init_kind != DECO_INIT_IDI && sp->init_kind != DECO_INIT_DUI && sp->init_kind != DECO_INIT_UNIFORM &&
      !(sp->init_kind == DECO_INIT_LEARNED && sp->magnitude))
    return DECO_E_INVAL;
  if (!supported_B(sp->B)) return DECO_E_UNSUPPORTED;
  deco_solver* v = new deco_solver();
  v->g = *g;
  v->p = *sp;
  v->p.eq0 = v->p.el0 = nullptr;
  v->p.l0 = nullptr;
  v->p.target_cut = nullptr;
  v->s = reinterpret_cast<hipStream_t>(stream);
  v->B = sp->B;
  v->K = sp->K;
  v->per = sp->B / sp->K;
  v->G = g->num_graphs;
  v->lmax = sp->l_max;
  v->NBY = nby_of(sp->B);
  v->n = g->n;
  deco_params pq{};
  pq.B = v->B;
  pq.l = 1;
  pq.lifted = 0;
  pq.grad_form = sp->grad_form;
  pq.x_dtype = sp->x_dtype;
  pq.score_every = 1;
  pq.eta = 0.1f;
  pq.seed = sp->seed;
  deco_params pl = pq;
  pl.l = v->lmax;
  pl.lifted = 1;
  size_t wq = 0, wl = 0;
  if ((st = deco_workspace_size(g, &pq, &wq)) || (st = deco_workspace_size(g, &pl, &wl))) {
    delete v;
    return st;
  }
  const size_t es = elem_size(sp->x_dtype);
  const size_t xq_b = align_up((size_t)v->n * v->B * es), xl_b = align_up((size_t)v->n * v->lmax * v->B * es);
  const size_t total = xq_b + xl_b + align_up(wq) + align_up(wl) + align_up((size_t)v->n);
  if (hipMalloc(&v->mem, total) != hipSuccess) {
    v->mem = nullptr;
    solver_free(v);
    return DECO_E_NOMEM;
  }
  char* xq = v->mem;
  char* xl = xq + xq_b;
  char* wsq = xl + xl_b;
  char* wsl = wsq + align_up(wq);
  v->mean_dev = reinterpret_cast<uint8_t*>(wsl + align_up(wl));
  if ((st = deco_init(&v->hq, g, &pq, xq, wsq, wq, stream)) || (st = deco_init(&v->hl, g, &pl, xl, wsl, wl, stream))) {
    solver_free(v);
    return st;
  }
  if (sp->autotune) {
    // shapes tuned earlier in this process already run their cached winner; resident
    // candidates are timed over calls as long as the run's own (a target check or a whole
    // batch, 10 to 1000 steps), so their fixed cost per call is judged at its real share
    const int call = sp->check_every > 0 ? sp->check_every : std::max(sp->T_q, sp->T_l);
    const int tune = std::max(10, std::min(1000, call));
    if ((!schedule_cached(v->hq) && (st = deco_autotune(v->hq, tune))) ||
        (!schedule_cached(v->hl) && (st = deco_autotune(v->hl, tune)))) {
      solver_free(v);
      return st;
    }
  }
  const int K = v->K;
  v->eq.resize(K);
  v->el.resize(K);
  v->lk.resize(K);
  v->tq.resize(K);
  v->tl.resize(K);
  // initial population drawn from the bounds (Sec. 4.3); explicit genes override the draw
  if ((st = deco_evo_init(K, -4.0, -1.0, v->lmax, sp->T_min > 0 ? sp->T_min : sp->T_q, sp->T_q,
                          sp->T_l_min > 0 ? sp->T_l_min : sp->T_l, sp->T_l, sp->seed, v->eq.data(), v->el.data(),
                          v->lk.data(), v->tq.data(), v->tl.data()))) {
    solver_free(v);
    return st;
  }
  for (int k = 0; k < K; ++k) {
    if (sp->eq0) v->eq[k] = sp->eq0[k];
    if (sp->el0) v->el[k] = sp->el0[k];
    if (sp->l0) v->lk[k] = std::min(v->lmax, std::max(1, sp->l0[k]));
  }
  if (sp->target_cut) v->target.assign(sp->target_cut, sp->target_cut + v->G);
  v->bc.resize((size_t)v->G * v->B);
  v->bits.resize((size_t)v->n * v->NBY);
  v->zmean.assign((size_t)v->n, 0);
  v->best_z.assign((size_t)v->n, 0);
  v->gbest.assign(v->G, -INFINITY);
  v->fit.resize(K);
  v->fitg.resize((size_t)K * v->G);
  v->eta.resize(v->B);
  v->lact.resize(v->B);
  v->goff.assign(v->G + 1, 0);
  if (g->graph_row_offset) {
    if (hipMemcpy(v->goff.data(), g->graph_row_offset, sizeof(int) * (v->G + 1), hipMemcpyDeviceToHost) !=
        hipSuccess) {
      solver_free(v);
      return DECO_E_DEVICE;
    }
  } else {
    v->goff[1] = (int)v->n;
  }
  *out = v;
  return DECO_OK;
}

deco_status deco_solver_run(deco_solver* v, int32_t rounds, double* best_cut, uint8_t* best_z, double* round_time,
                            double* round_best, deco_solve_report* report) {
  if (!v || rounds < 0) return DECO_E_INVAL;
  const double t_start = now_s();
  const deco_solve_params& sp = v->p;
  const int B = v->B, K = v->K, G = v->G;
  deco_status st;
  int done_here = 0;
  for (int rr = 0; rr < rounds; ++rr) {
    const int r = v->round;
    std::fill(v->fitg.begin(), v->fitg.end(), -INFINITY);
    // the first batch of the run starts from the chosen start, every later one is centred on
    // the previous batch's best vector (Sec. 4.2)
    bool first = r == 0;
    deco_start_args sa{};
    sa.mean_z = v->mean_dev;
    sa.magnitude = sp.magnitude;
    sa.sigma2 = sp.sigma2;
    sa.beta = sp.beta;
    bool hit = false;
    if (sp.mode != DECO_SOLVE_LIFTED) {
      // 1. unlifted batch (Alg. 1): member k's columns step with 10^eq[k]
      for (int b = 0; b < B; ++b) v->eta[b] = (float)std::pow(10.0, v->eq[b / v->per]);
      if ((st = deco_set_eta(v->hq, v->eta.data()))) return st;
      sa.kind = first ? sp.init_kind : DECO_INIT_MEAN;
      sa.scale = (sp.init_kind == DECO_INIT_UNIFORM && first) ? 1.0 : sp.scale;
      sa.batch = v->batch++;
      if ((st = deco_start(v->hq, &sa))) return st;
      first = false;
      int tmax = 0;
      if ((st = run_counts(v, v->hq, v->eta, v->tq, &tmax, &hit))) return st;
      if ((st = deco_round_score(v->hq, nullptr, nullptr))) return st;
      if ((st = absorb(v, v->hq))) return st;
      v->steps_done += tmax;
      // edge updates of the members' own steps (a member past its count keeps still)
      for (int k = 0; k < K; ++k) v->eu += (double)v->g.nnz * v->per * std::min(v->tq[k], tmax);
    }
    // 2. lift its best vector (Alg. 3 step 2) and run the lifted batch (Alg. 2); member k
    //    keeps lk[k] of the lmax components and steps with 10^el[k]; 3. project back
    if (!hit && sp.mode != DECO_SOLVE_UNLIFTED) {
      for (int b = 0; b < B; ++b) {
        v->eta[b] = (float)std::pow(10.0, v->el[b / v->per]);
        v->lact[b] = v->lk[b / v->per];
      }
      if ((st = deco_set_eta(v->hl, v->eta.data()))) return st;
      sa.kind = first ? sp.init_kind : DECO_INIT_MEAN;
      sa.scale = (sp.init_kind == DECO_INIT_UNIFORM && first) ? 1.0 : sp.scale;
      sa.batch = v->batch++;
      sa.l_active = v->lact.data();
      if ((st = deco_start(v->hl, &sa))) return st;
      int tlmax = 0;
      if ((st = run_counts(v, v->hl, v->eta, v->tl, &tlmax, &hit))) return st;
      if ((st = deco_round_score(v->hl, nullptr, nullptr))) return st;
      if ((st = absorb(v, v->hl))) return st;
      v->steps_done += tlmax;
      // active components only: components past a member's lift dimension stay exactly 0
      for (int k = 0; k < K; ++k) v->eu += (double)v->g.nnz * v->per * v->lk[k] * std::min(v->tl[k], tlmax);
    }
    for (int k = 0; k < K; ++k) {
      v->fit[k] = 0.0;
      for (int gi = 0; gi < G; ++gi) v->fit[k] += v->fitg[(size_t)k * G + gi];
    }
    if (round_time) round_time[rr] = now_s() - t_start;
    if (round_best)
      for (int gi = 0; gi < G; ++gi) round_best[(size_t)rr * G + gi] = v->gbest[gi];
    // 4. evolutionary search between batches (Sec. 4.3)
    if (r < sp.evo_rounds) {
      std::vector<double> q(K), m(K);
      std::vector<int32_t> ll(K);
      if ((st = deco_evo_next(K, v->fit.data(), v->eq.data(), v->el.data(), v->lk.data(), -4.0, -1.0, v->lmax,
                              sp.seed, (uint32_t)r, q.data(), m.data(), ll.data())))
        return st;
      if (sp.T_min > 0) {
        std::vector<int32_t> tt(K);
        if ((st = deco_evo_next_steps(K, v->fit.data(), v->tq.data(), sp.T_min, sp.T_q, sp.seed, (uint32_t)r, 0,
                                      tt.data())))
          return st;
        v->tq = tt;
      }
      if (sp.T_l_min > 0) {
        std::vector<int32_t> tt(K);
        if ((st = deco_evo_next_steps(K, v->fit.data(), v->tl.data(), sp.T_l_min, sp.T_l, sp.seed, (uint32_t)r, 1,
                                      tt.data())))
          return st;
        v->tl = tt;
      }
      v->eq = q;
      v->el = m;
      v->lk = ll;
      if (r == sp.evo_rounds - 1)
        for (int k = 1; k < K; ++k) {
          v->eq[k] = v->eq[0];
          v->el[k] = v->el[0];
          v->lk[k] = v->lk[0];
          v->tq[k] = v->tq[0];
          v->tl[k] = v->tl[0];
        }
    }
    v->round++;
    done_here++;
    bool stop = hit || (sp.time_budget_s > 0 && now_s() - t_start >= sp.time_budget_s);
    if (!v->target.empty()) {
      bool all = true;
      for (int gi = 0; gi < G; ++gi) all = all && v->gbest[gi] >= v->target[gi];
      stop = stop || all;
    }
    if (stop) break;
  }
  if (best_cut)
    for (int gi = 0; gi < G; ++gi) best_cut[gi] = v->gbest[gi];
  if (best_z) std::memcpy(best_z, v->best_z.data(), (size_t)v->n);
  if (report) {
    report->rounds_done = done_here;
    report->steps_done = v->steps_done;
    report->edge_updates = v->eu;
    report->seconds = now_s() - t_start;
    report->eq_best = v->eq[0];
    report->el_best = v->el[0];
    report->l_best = v->lk[0];
    report->T_best = v->tq[0];
    report->T_l_best = v->tl[0];
  }
  return DECO_OK;
}

deco_status deco_solver_set_target(deco_solver* v, const double* target_cut) {
  if (!v) return DECO_E_INVAL;
  if (target_cut)
    v->target.assign(target_cut, target_cut + v->G);
  else
    v->target.clear();
  return DECO_OK;
}

void deco_solver_destroy(deco_solver* v) { solver_free(v); }

deco_status deco_solve(const deco_graph* g, const deco_solve_params* sp, void* stream, double* best_cut,
                       uint8_t* best_z, double* round_time, double* round_best, deco_solve_report* report) {
  if (!sp || !best_cut || !best_z) return DECO_E_INVAL;
  if (sp->rounds < 1) return DECO_E_INVAL;
  const double t0 = now_s();
  deco_solver* v = nullptr;
  deco_status st = deco_solver_create(&v, g, sp, stream);
  if (st) return st;
  st = deco_solver_run(v, sp->rounds, best_cut, best_z, round_time, round_best, report);
  if (!st && report) report->seconds = now_s() - t0;
  solver_free(v);
  return st;
}

}  // extern "C"
