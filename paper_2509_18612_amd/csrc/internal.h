// Internal interface between the host side (api.hip) and the kernels (kernels.hip) of the
// DECO library. Not installed; the public ABI is include/deco.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace deco {

// Device-resident control block of one handle. The step kernels read it at their start
// and the last workgroup of every step updates it, so a captured graph of step launches
// can be replayed without host involvement.
//
// Scoring of step t runs in three stages: launch t accumulates the score sums of X_t into
// acc[t & 1] and writes its cut bits into bits[t % 3]; the completion of step t (sums to
// cuts, best cut and step, improvement mask into mask[t & 1]) runs either in the last
// workgroup of launch t (immediate mode) or in extra workgroups of launch t + 1 (lagged
// mode, off the critical path); the launch after the completion folds the improved bits
// into best_bits. A drain (launch_drain) completes and folds whatever is pending, so the
// results are current after every host call that runs steps.
struct DevCtrl {
  unsigned int ticket;  // XCDs whose workgroups all finished the current launch
  int score_every;
  long long t;          // index of the current iterate
  long long cpend;      // scored step whose completion is pending (-1: none)
  long long fpend;      // completed step whose improvements are not yet folded (-1: none)
  long long drain[2];   // steps the drain folds, in this order (-1: none)
  unsigned int xticket[8][64];  // per-XCD completion counters, 256 bytes apart
};

// Work-item limits of the step kernel (LDS staging of one item's slot list).
constexpr int kEmax = 2048;  // slots staged at a time
constexpr int kRmax = 512;   // rows of a normal item
constexpr int kMaxL = 8;     // lifted components per initialisation held by one step kernel
                             // (more run as a pair of handles, see api.hip)

// Slot list: row v occupies positions [row_ptr[v] + v, row_ptr[v+1] + v + 1): its own
// index with the top bit set, then its neighbours in CSR order. The slot weights (weighted
// graphs) hold the weighted degree at the row's own position and w_vu after it.
//
// One work item is two int4: {x, y, s0, s1} = rows [x, y) and their slots [s0, s1), then
// {graph, initialisation tile, long-row flag, 0}; a long-row item is a single row handled
// by the whole workgroup. Items are grouped by XCD: items[seg[x] .. seg[x+1]) run on
// workgroups with blockIdx % 8 == x.

struct StepArgs {
  const int* rp;
  const int* ci;
  const float* w;   // NULL = unit weights
  const float* dw;  // weighted degree (Laplacian form), may be NULL for the cut form
  void* x[2];       // ping-pong iterates; x[t & 1] holds X_t
  int C, B, lifted;
  int L;            // components per initialisation the step kernel runs: the handle's l, or the
                    // largest active count when that is smaller (the components past it are 0 in
                    // both iterate buffers and no kernel writes them)
  int Wc;           // lanes per row team (power of two, <= 64; Wc * VEC <= 256)
  const int* slots; // slot list (n + nnz)
  const float* sw;  // slot weights (n + nnz), NULL for unit weights
  const int4* items;
  const int* seg;   // [9]
  float cW, cD;     // G = cW * (W X) + cD * (d_w . X)
  const float* eta; // [B]
  const int* lact;  // [B] active components of each initialisation (components at and past
                    // it are exactly 0 in X and are not gathered), or NULL (all l active)
  uint8_t* bits[3]; // cut bits of the iterate scored at step t live in bits[t % 3]
  uint8_t* best_bits;
  uint8_t* mask;    // [2][G][NBY]: improvements of scored step t in mask[t & 1]
  int NBY;
  double* acc;      // [2][R][G][B] partial sums of w 1{z_v != z_u}; step t uses acc[t & 1]
  int R, G;
  int nextra;       // lagged mode: workgroups after the work grid that complete step t - 1
                    // (0: immediate mode)
  float* vel;       // heavy-ball velocity, float32 n x C (same layout as X), or NULL
  float mu;         // momentum coefficient (with vel)
  double* cur_cut;  // [G][B]
  double* best_cut; // [G][B]
  int* best_step;   // [G][B]
  double* trace;    // optional [trace_cap][G][B]
  int trace_cap;
  DevCtrl* ctrl;
  int do_update;    // 0: score-only pass (no new iterate, step counter unchanged)
  int force_score;  // score this launch regardless of score_every
  int intw;         // all weights are integers of magnitude <= 1024 (int32 score partials)
  int pm1;          // all weights are +-1
  double cut_scale; // cut = cut_scale * accumulated sum (1/2 sparse path, 1/4 dense path)
  const uint16_t* dense_w;  // dense path: bfloat16 n x n weight matrix (row-major)
  void* xT[2];              // dense path: transposed iterates (C x n); xT[t & 1] holds X_t^T
  long long n;      // rows
};

// Kernel launchers (kernels.hip). dtype: 0 float32, 1 bfloat16. vec: elements per lane
// per load (native_vec, or 1).
hipError_t launch_step(const StepArgs& a, int dtype, int vec, int grid, hipStream_t s);
// The same for handles with a velocity (a.vel != NULL): the kernels with the heavy-ball
// update (step_momentum.hip).
hipError_t launch_step_momentum(const StepArgs& a, int dtype, int vec, int grid, hipStream_t s);
// Step kernels of 5..8 lifted components (plain; routes momentum to the second launcher).
hipError_t launch_step_wide(const StepArgs& a, int dtype, int vec, int grid, hipStream_t s);
hipError_t launch_step_wide_momentum(const StepArgs& a, int dtype, int vec, int grid, hipStream_t s);
int native_vec(int dtype, int L);
// Dense path: n % 128 == 0, C % 128 == 0, bfloat16 X and W, unlifted.
hipError_t launch_dense_step(const StepArgs& a, hipStream_t s);
// XT = X^T (bfloat16 n x C -> C x n); n % 64 == 0, C % 64 == 0.
hipError_t launch_dense_transpose(const void* X, void* XT, long long n, int C, hipStream_t s);
hipError_t launch_dense_validate(const uint16_t* W, int n, float* dw, int* flags, hipStream_t s);

hipError_t launch_validate(long long n, const int* rp, const int* ci, const float* w,
                           const int* goff, int G, float* dw, int* flags, hipStream_t s);
// Builds the slot list (and slot weights when w != NULL) of a validated graph.
hipError_t launch_build_slots(long long n, long long nnz, const int* rp, const int* ci, const float* w,
                              const float* dw, int* slots, float* sw, hipStream_t s);
hipError_t launch_reset(StepArgs a, double* acc_all, long long acc_count, int score_every,
                        hipStream_t s);
hipError_t launch_merge(StepArgs a, long long n, const int* goff, hipStream_t s);
// Completes a pending scored step and folds the pending improvements into best_bits
// (two launches); idempotent.
hipError_t launch_drain(StepArgs a, long long n, const int* goff, hipStream_t s);
// Workgroups that complete one step's G * B cuts (256 each, at most 64).
int completion_blocks(long long GB);
hipError_t launch_fill_eta(float* eta, int B, float v, hipStream_t s);
// Zeroes 'bytes' bytes (an even count) of device memory with a kernel.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
// Resident steps (resident.hip): 'steps' steps of an unlifted (or l = 1) batch in one launch,
// one workgroup per item {graph, first row, end row, first column} holding bt columns of the
// graph's rows in LDS; then the step counter advances by 'steps'. prepare_resident raises the
// kernels' LDS limit once per schedule (outside stream capture).
// The slots of each graph are split into equal shares over resident_threads(bt) threads and
// read from an interleaved stream (build_resident_stream, once per schedule: 4 ints of header
// per thread, then the slots): rgs[g] = {stream offset, slots per thread rounded up to 4,
// slots E_g, first slot of graph g}.
int resident_threads(int bt);
size_t resident_lds_bytes(int max_rows, int bt, int dtype);
hipError_t prepare_resident(const StepArgs& a, int dtype, int bt, int max_rows);
hipError_t build_resident_stream(long long nslots, int G, int bt, const int4* rgs, const int* goff, const int* rp,
                                 const int* slots, const float* sw, int* stream, float* wstream, hipStream_t s);
// rbest (B / bt byte arrays of n rows) and rimp (G x B / bt flags) carry the best sides of
// tiles narrower than 8 columns to a merge kernel after the launch.
hipError_t launch_resident(const StepArgs& a, int dtype, int bt, const int4* items, int nitems, const int4* rgs,
                           const int* stream, const float* wstream, uint8_t* rbest, uint8_t* rimp, const int* goff,
                           int max_rows, int steps, hipStream_t s);
// Component sums of a many-component batch (l > kMaxL) into the score handle's iterate.
hipError_t launch_sides(const void* x0, const void* x1, void* s0, void* s1, const DevCtrl* cx, const DevCtrl* cs,
                        long long n, int B, int l, int dtype, hipStream_t s);

struct InitArgs {
  long long n;
  int C, B, L;
  const int* rp;
  const int* ci;
  const float* w;
  const int* goff;   // [G+1] device
  int G;
  const double* thr; // IDI threshold per graph [G]
  const int* delta;  // max degree per graph [G]
  const uint8_t* mean_z;
  const int* l_active; // device [B] or NULL
  const float* magnitude; // learned magnitudes [n] or NULL
  int8_t* scratch;   // n*C bytes (IDI important signs)
  double scale, sd;
  unsigned long long seed;
  unsigned batch;
  int kind;
  int dtype;
  void* X;
};
hipError_t launch_init(const InitArgs& a, hipStream_t s);
hipError_t launch_convert_user(const void* x0, void* X, long long count, int dtype,
                               const int* l_active, int C, int B, int* nonfinite,
                               hipStream_t s);
hipError_t launch_philox_test(uint32_t c1, uint32_t c2, uint32_t c3, unsigned long long seed,
                              int count, uint32_t* out, hipStream_t s);

// Counter-based generator shared by host and device code of the library.
__host__ __device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
  }
}

enum Purpose : uint32_t { kUniform = 1, kDui = 2, kIdiSign = 3, kIdiTie = 4, kGauss = 5, kSearch = 6 };

}  // namespace deco
