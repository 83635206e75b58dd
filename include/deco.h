/*
 * deco.h - C ABI of the MI355X (gfx950) DECO library: batched projected gradient ascent
 * for MaxCut on the relaxed quadratic objectives of Alkhouri et al., "A Scalable
 * Lift-and-Project Differentiable Approach For the Maximum Cut Problem".
 *
 * The hot path is the batched gradient step (Sec. 3.1 eq. (6)-(7); Sec. 3.2 lifted
 * update), the roundings to a cut (eq. (5); Sec. 3.2 lifted rounding), the exact cut of
 * eq. (1) and the running best over iterates (Alg. 1 and 2, steps 4-6). DECO (Alg. 3)
 * alternates it between the unlifted and lifted formulations from an importance-based
 * degree start (Sec. 4.1), with the evolutionary step-size search of Sec. 4.3.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Graph: symmetric CSR storing both directions of every undirected edge, rows sorted by
 *   column, no self-loops, no duplicates; weights w_uv = w_vu (NULL = unit weights, the
 *   paper's adjacency A). Several graphs may be stacked block-diagonally; graph g owns rows
 *   [graph_row_offset[g], graph_row_offset[g+1]) and has no edge leaving them.
 *   All graph arrays are DEVICE pointers owned by the caller; they must stay valid and
 *   unchanged while a handle that uses them exists.
 * Batch: every graph carries B initialisations; in lifted mode each has l components.
 *   X is an n x (l*B) row-major DEVICE array (float32 or bfloat16 storage) in which node v,
 *   component i, initialisation b sits at X[v*l*B + i*B + b] ("component-major").
 * Cut bits: z_v(b) of row v is bit (b % 8) of byte X_bits[v*nby + b/8], nby = ceil(B/8).
 * Results per (graph g, initialisation b) are stored at index g*B + b.
 * Gradient forms: DECO_GRAD_CUT (default) uses G = -1/2 W X, the exact gradient of
 *   F(x) = 1/2 sum_{(u,v) in E} w_uv (1 - x_u x_v), which equals the cut on {-1,1}^n;
 *   DECO_GRAD_LAPLACIAN uses G = L X = D_w X - W X exactly as eq. (6) prints it.
 * Rounding: unlifted z_v = 1{x_v > 0} (eq. (5)); lifted z_v = 1{sum_i X[v,i,b] >= 0} with
 *   the sum formed in float32 in component order (Sec. 3.2).
 * Exact cut: sum over rows of w_vu 1{z_v != z_u}, halved. Integer weights of magnitude
 *   <= 1024 (unit and +-1 included) are summed in int32 per work item and double across
 *   items, so the cut is exact and order-free (below 2^53). Other weights use float32 per
 *   item (at most 2048 terms per partial), then double: |error| <= sum|w| * 2^-14.
 *
 * Errors: every function returns a deco_status. Arguments are validated before anything
 * is launched, so an error return has no side effect on the device. An asynchronous
 * device fault is reported as DECO_E_DEVICE by the next call that synchronises; the
 * handle is then poisoned and later calls on it return DECO_E_STATE. Nothing throws or
 * aborts across the ABI. A handle is not thread-safe; different handles are independent.
 * Streams: 'stream' arguments are hipStream_t values passed as void*; NULL is the
 * default stream. All work of a handle is ordered on its stream.
 */
#ifndef DECO_H
#define DECO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t deco_status;
#define DECO_OK 0
#define DECO_E_INVAL (-1)       /* bad argument, bad graph structure or bad sizes */
#define DECO_E_NOMEM (-2)       /* caller workspace too small, or allocation failed */
#define DECO_E_DEVICE (-3)      /* HIP runtime or kernel error */
#define DECO_E_STATE (-4)       /* handle poisoned by an earlier device error */
#define DECO_E_NONFINITE (-5)   /* NaN or Inf in weights or starting values */
#define DECO_E_UNSUPPORTED (-6) /* shape outside what the kernels handle (see below) */

#define DECO_GRAD_CUT 0
#define DECO_GRAD_LAPLACIAN 1

#define DECO_F32 0
#define DECO_BF16 1

/* Starting points (Sec. 4.1, Sec. 4.2 and the down-scaling of Sec. 5). */
#define DECO_INIT_USER 0    /* copy x0 (device, n x l*B, storage dtype) */
#define DECO_INIT_UNIFORM 1 /* x = 2u - 1, u uniform on the 2^-24 grid of [0,1) */
#define DECO_INIT_DUI 2     /* mean h ~ U[-(1-d_v/Delta), 1-d_v/Delta] per column */
#define DECO_INIT_IDI 3     /* mean h = importance-based signs per column */
#define DECO_INIT_MEAN 4    /* mean h = 2 z - 1 from a device byte vector z[n] */
#define DECO_INIT_LEARNED 5 /* mean h = y_v * IDI sign (y: device float magnitudes[n], e.g. from
                               deco_mpnn_forward) */

/* Random draws: Philox4x32-10 (Salmon et al., SC'11) with key = (seed low, seed high)
 * and counter = (row, column, purpose, batch); purposes 1 uniform, 2 DUI, 3 IDI sign,
 * 4 IDI tie coin, 5 Gaussian, 6 search. u = (r >> 8) * 2^-24; Gaussian by Box-Muller
 * eps = sqrt(-2 ln u1) cos(2 pi u2) with u1 = ((r0 >> 8) + 1) 2^-24, u2 = (r1 >> 8) 2^-24. */

typedef struct deco_graph {
  int64_t n;                       /* total rows (sum over stacked graphs), >= 1 */
  int64_t nnz;                     /* stored entries (2 x undirected edges), < 2^31 */
  const int32_t *row_ptr;          /* device [n+1] */
  const int32_t *col_idx;          /* device [nnz] */
  const float *w;                  /* device [nnz], or NULL for unit weights */
  int32_t num_graphs;              /* >= 1 */
  const int32_t *graph_row_offset; /* device [num_graphs+1]; NULL allowed when num_graphs == 1 */
} deco_graph;

typedef struct deco_params {
  int32_t B;            /* initialisations per graph: 1, 2, 4 or a multiple of 8 */
  int32_t l;            /* components per initialisation (1 = unlifted), up to l*B < 2^24; at
                           most 8 are held by one step kernel, more run as an unlifted handle
                           over the l*B columns (the lifted update acts column by column)
                           plus a lifted l = 1 handle scoring the float32 component sums, with
                           identical results (the workspace holds both) */
  int32_t lifted;       /* 0: eq. (5) rounding (requires l == 1); 1: lifted rounding */
  int32_t grad_form;    /* DECO_GRAD_CUT or DECO_GRAD_LAPLACIAN */
  int32_t x_dtype;      /* DECO_F32 or DECO_BF16 storage of X (arithmetic is float32) */
  int32_t score_every;  /* score iterate t when t % score_every == 0 (>= 1) */
  float eta;            /* step size (the paper's alpha) for every initialisation */
  uint64_t seed;        /* key of the counter-based generator */
} deco_params;

typedef struct deco_start_args {
  int32_t kind;            /* DECO_INIT_* */
  const void *x0;          /* USER: device n x l*B array in the storage dtype */
  const uint8_t *mean_z;   /* MEAN: device [n] bytes in {0,1} */
  double scale;            /* starting values are divided by 'scale' (Sec. 5 uses 1e4); >0 */
  double sigma2;           /* variance of the Gaussian exploration noise around the mean
                              (Sec. 4.2, the paper's eta); 0 = no noise. Not used by
                              USER and UNIFORM. */
  double beta;             /* IDI threshold factor (Sec. 4.1, default 0.2) */
  uint32_t batch;          /* batch index in the generator's counter */
  const int32_t *l_active; /* host [B] or NULL: components i >= l_active[b] of
                              initialisation b start at exactly 0 (and stay 0) */
  const float *magnitude;  /* LEARNED: device [n] per-node magnitudes */
} deco_start_args;

typedef struct deco_handle deco_handle;

/* Human-readable name of a status code (static string, never NULL). */
const char *deco_status_string(deco_status s);

/* Device workspace (bytes) a handle for (g, p) needs; host-only, no device access
 * except reading nothing: the size depends only on n, nnz, num_graphs and p. */
deco_status deco_workspace_size(const deco_graph *g, const deco_params *p, size_t *bytes);

/* Validate the graph on the device (structure, symmetry, finite weights; synchronous),
 * build the row/column schedule and bind the caller's X (device, n x l*B, 16-byte
 * aligned) and workspace (device, >= deco_workspace_size bytes, 256-byte aligned).
 * The handle is small host memory owned by the library (free with deco_destroy).
 * Errors: DECO_E_INVAL (structure), DECO_E_NONFINITE (weights), DECO_E_NOMEM
 * (workspace), DECO_E_UNSUPPORTED (B or l outside the supported set, nnz >= 2^31). */
deco_status deco_init(deco_handle **out, const deco_graph *g, const deco_params *p, void *X,
                      void *workspace, size_t workspace_bytes, void *stream);

/* Fill the current iterate per 'a' (Sec. 4.1-4.2) and reset the running best
 * (best cut -inf, step -1) and the step counter to 0. Asynchronous. */
deco_status deco_start(deco_handle *h, const deco_start_args *a);

/* Set a per-initialisation step size (host eta[B]); replaces deco_params.eta. */
deco_status deco_set_eta(deco_handle *h, const float *eta_host);

/* Heavy-ball momentum for the following steps (Sec. 4.2 runs PGA with momentum, Sec. 5 with
 * coefficient 0.9; the paper gives no update rule, this is the heavy-ball reading):
 * V' = mu V + G, X' = Proj(X + eta V'). velocity: device float32 n x (l*B), the layout of X,
 * caller-owned, zeroed by this call and by every deco_start (a start begins at rest); the
 * library reads and writes it at every step. NULL turns momentum off. Sparse handles only
 * (DECO_E_UNSUPPORTED on dense ones); DECO_E_NONFINITE for a non-finite mu. Synchronous. */
deco_status deco_set_momentum(deco_handle *h, float mu, float *velocity);

/* Run 'steps' projected gradient steps (eq. (7) / the lifted update) on the handle's
 * stream, asynchronously, with no host synchronisation. Step t scores the iterate X_t it
 * reads (when t % score_every == 0) and folds it into the running best; X_steps is left
 * unscored until the next step or deco_round_score. Inside the call a step's cuts are
 * completed by the following launch; the call ends with a drain (two small kernels), so
 * the cuts, trace, running best and best bits of every step it ran are complete on the
 * stream when the next operation on it starts. With use_graph != 0 the step launches are
 * captured once per step count into a hipGraph and replayed (the stream must not be the
 * NULL stream then); the drain runs after the replay. */
deco_status deco_step(deco_handle *h, int32_t steps, int32_t use_graph);

/* Round and score the current iterate exactly (eq. (5) or the lifted rule, then eq. (1)),
 * fold it into the running best, and optionally export the cuts (device double [G*B])
 * and the cut bits (device bytes [n*nby]). Asynchronous. */
deco_status deco_round_score(deco_handle *h, double *cut_out, uint8_t *bits_out);

/* Synchronise and copy the running best to HOST memory: best cut per (g, b) [G*B],
 * step at which it was reached [G*B] (may be NULL), and the best cut bits [n*nby]
 * (may be NULL). */
deco_status deco_best(deco_handle *h, double *best_cut, int32_t *best_step, uint8_t *best_bits);

/* Copy the current iterate (n x l*B, storage dtype) to a device buffer. Asynchronous. */
deco_status deco_read_x(deco_handle *h, void *dst);

/* Optional per-step cut trace: after this call every scored step t writes its cuts to
 * trace[(t % capacity) * G*B + g*B + b] (device doubles). NULL disables it. */
deco_status deco_set_trace(deco_handle *h, double *trace, int32_t capacity);

/* Index of the current iterate (number of steps taken since deco_start). Host-side. */
int64_t deco_current_step(const deco_handle *h);

/* Choose the kernel schedule (b-tile width, long-row threshold, work item size, XCD layout,
 * or the resident schedule for unlifted and l = 1 handles) by timing candidates on the
 * device and comparing their time per step: resident schedules over a call of 'steps'
 * steps (they have a fixed cost per call, so 'steps' should be the length of the calls that
 * will follow), step-kernel schedules over min(steps, 50) steps; the winner is kept in the
 * handle and in a per-process cache keyed by the graph and batch shape. It overwrites X
 * and the running best (call deco_start afterwards). Synchronous. */
deco_status deco_autotune(deco_handle *h, int32_t steps);

/* Set the kernel schedule explicitly (instead of the default or the autotuner's choice).
 * lanes_per_row: lanes of one row team, which holds one row's initialisation tile (power
 * of two <= 64; the tile is lanes_per_row * (16 bytes / element size) columns, 8 bytes for
 * lifted bfloat16 and for float32 handles of l = 2..8; it must divide B, hold at most 256 columns, and at least 64 when 64
 * divides B for unlifted handles, 16 when 16 divides B for lifted ones); long_row: rows with more neighbours get a work item of their own (>= 16; rows
 * with more slots than nnz_per_item always do); xcd_mode: 0 = each XCD owns a row range
 * for every tile, 1 = each XCD owns tiles; blocks_per_xcd: workgroups per XCD (1..4096;
 * with more items than workgroups a workgroup walks several); nnz_per_item: target slots
 * (edges plus rows) per work item (128..2048); lane_elems: 0 = the native lane width, or
 * 4 = four values per lane: for unlifted bfloat16 rows (8-byte loads, twice the lanes per
 * tile) and for float32 handles of l = 2..8 (16-byte loads, half the lanes per tile), or
 * 2 = two values per lane for bfloat16 handles of l = 2..8 (4-byte loads, twice the lanes). DECO_E_INVAL when the values do not fit B or the limits.
 * Synchronous (uploads the work list). */
typedef struct deco_schedule {
  int32_t lanes_per_row, long_row, xcd_mode, blocks_per_xcd, nnz_per_item, lane_elems;
  int32_t resident_cols; /* > 0: resident steps (unlifted or l = 1 handles): every step of a
                            deco_step call in one launch, one workgroup per (graph, tile of
                            resident_cols columns) holding that tile of the graph's rows in
                            LDS for all the steps (1, 2, 4, 8 or 16 dividing B; the graph's
                            rows plus 64 spare rows times the tile, two buffers, must fit one
                            workgroup's LDS, else DECO_E_UNSUPPORTED; the graph's slots are
                            split evenly over 1024, 512 or 256 threads for tiles of 1, 2 or
                            more columns); score-only passes and momentum steps
                            keep the step kernel with its default schedule (the other fields
                            are not used then). 0: the step kernel with the fields above */
} deco_schedule;
deco_status deco_set_schedule(deco_handle *h, const deco_schedule *s);

/* ---------------------------------------------------------------------------------
 * Dense graphs (same method, Sec. 3.1 eq. (6)-(7) with a dense W): the gradient W X is a
 * GEMM on the bfloat16 matrix cores with float32 accumulation, and the exact cut comes from
 * the same GEMM against the sign matrix S = 2Z - 1: cut_b = 1/4 sum_v (d_w(v) - s_v (W s)_v).
 * The weights must be integers whose magnitudes sum to at most 2^24 in every row: then every
 * entry of W s and d_w is an exact float32 integer, the per-column sums are formed in double,
 * and the cut is exact. W: device bfloat16 n x n, row-major, symmetric, zero diagonal,
 * caller-owned. Requires n % 128 == 0, B % 128 == 0, l == 1 (unlifted), x_dtype ==
 * DECO_BF16 and the weight condition above; otherwise DECO_E_UNSUPPORTED. The handle then works with deco_start (USER, UNIFORM and MEAN
 * starts), deco_set_eta, deco_step, deco_round_score, deco_best, deco_read_x,
 * deco_set_trace and deco_destroy. deco_dense_init validates W on the device
 * (symmetry, diagonal, finiteness: DECO_E_INVAL / DECO_E_NONFINITE).
 * --------------------------------------------------------------------------------- */
deco_status deco_dense_workspace_size(int64_t n, const deco_params *p, size_t *bytes);
deco_status deco_dense_init(deco_handle **out, int64_t n, const void *W, const deco_params *p, void *X,
                            void *workspace, size_t workspace_bytes, void *stream);

/* Describe the schedule in use (NUL-terminated text into buf[cap]). */
deco_status deco_schedule_string(const deco_handle *h, char *buf, int32_t cap);

/* Release the handle (host memory only; caller-owned device memory is untouched). */
void deco_destroy(deco_handle *h);

/* ---------------------------------------------------------------------------------
 * Full pDECO (Alg. 3) with the evolutionary search of Sec. 4.3, blocking.
 * Each round: an unlifted batch of T_q steps (columns split into K member groups with
 * step 10^eq[k]), a lift of its best vector to l_max components per initialisation
 * (member k keeps l[k] of them active) and a lifted batch of T_l steps with step
 * 10^el[k]; the lifted batch's best vector is the next round's mean (Sec. 4.2). The first
 * evo_rounds rounds evolve the population (rank, keep the top half, perturb it into the
 * bottom half); later rounds use the best member's genes everywhere. The loop stops after
 * 'rounds' rounds, when 'time_budget_s' (> 0) is spent, or when every graph's best
 * reaches target_cut[g] (if target_cut != NULL; checked after every round, or every
 * check_every steps). Allocates and frees its own device
 * memory. Outputs (HOST): best cut per graph [G], its bits z[n] (bytes in {0,1}),
 * per-round wall time since the start [rounds] and best cut per graph [rounds*G].
 * --------------------------------------------------------------------------------- */
#define DECO_SOLVE_DECO 0      /* lift-and-project rounds: an unlifted then a lifted batch (Alg. 3) */
#define DECO_SOLVE_UNLIFTED 1  /* unlifted batches only (pQUCO, Alg. 1, with the search) */
#define DECO_SOLVE_LIFTED 2    /* lifted batches only (pLUCO, Alg. 2, with the search) */

typedef struct deco_solve_params {
  int32_t B;            /* initialisations per graph (multiple of K) */
  int32_t K;            /* population size (column groups), >= 1 */
  int32_t l_max;        /* lifted components per initialisation, >= 1 (deco_params.l) */
  int32_t rounds;       /* maximum number of lift-and-project rounds */
  int32_t evo_rounds;   /* rounds during which the population evolves */
  int32_t T_q;          /* steps of every unlifted batch */
  int32_t T_l;          /* steps of every lifted batch */
  int32_t grad_form;    /* DECO_GRAD_* */
  int32_t x_dtype;      /* DECO_F32 or DECO_BF16 */
  int32_t init_kind;    /* DECO_INIT_IDI, DECO_INIT_DUI, DECO_INIT_UNIFORM or DECO_INIT_LEARNED
                           (with 'magnitude') for the first batch */
  double beta, sigma2, scale; /* Sec. 5: 0.2, 0.8, 1e4 */
  double time_budget_s; /* <= 0: no time limit */
  uint64_t seed;
  const double *eq0;    /* host [K]: initial log10 steps of the unlifted batch, or NULL (drawn
                           by deco_evo_init, Sec. 4.3) */
  const double *el0;    /* host [K]: initial log10 steps of the lifted batch, or NULL (drawn) */
  const int32_t *l0;    /* host [K]: initial lift dimensions, or NULL (drawn) */
  const double *target_cut; /* host [G] or NULL */
  int32_t use_graph;    /* capture the step loops in hipGraphs */
  int32_t autotune;     /* run deco_autotune on both handles first, over calls of the run's
                           own length (check_every, else the longer batch; 10 to 1000 steps); a
                           shape already tuned in this process reuses its cached winner */
  int32_t T_min;        /* > 0: the unlifted step count is searched per member in [T_min, T_q]
                           (Sec. 4.3: drawn uniformly, evolved by deco_evo_next_steps; a member
                           past its count keeps its columns still with a step of 0); 0: T_q */
  int32_t T_l_min;      /* > 0: the same for the lifted step count in [T_l_min, T_l]; 0: T_l */
  const float *magnitude; /* init_kind == DECO_INIT_LEARNED: device [n] per-node magnitudes
                             (e.g. from deco_mpnn_forward), read by the first batch of every
                             run of a solver, so it must stay valid while the solver exists;
                             NULL otherwise */
  int32_t check_every;  /* > 0 with target_cut: every batch also pauses every check_every steps
                           to compare the graphs' bests with their targets (one synchronisation
                           each) and the run ends as soon as every graph reached its target, in
                           the middle of a round if need be; 0: targets are checked after each
                           round */
  int32_t mode;         /* DECO_SOLVE_DECO (default 0), DECO_SOLVE_UNLIFTED or DECO_SOLVE_LIFTED:
                           which batches a round runs; the first batch of the run starts from
                           init_kind, later ones from the previous batch's best vector */
} deco_solve_params;

typedef struct deco_solve_report {
  int32_t rounds_done;
  int64_t steps_done;       /* gradient steps over all batches */
  double edge_updates;      /* sum over the members' own gradient steps of nnz * active
                               columns: B/K initialisations per member, times its lift
                               dimension in the lifted batch (inactive components and the
                               still steps of a member past its count are not counted) */
  double seconds;           /* wall time of the whole call */
  double eq_best, el_best;  /* genes of the best member at the end */
  int32_t l_best;
  int32_t T_best;           /* unlifted step count of the best member at the end */
  int32_t T_l_best;         /* lifted step count of the best member at the end */
} deco_solve_report;

deco_status deco_solve(const deco_graph *g, const deco_solve_params *p, void *stream,
                       double *best_cut, uint8_t *best_z, double *round_time,
                       double *round_best, deco_solve_report *report);

/* The same loop as a persistent object, for callers that solve in pieces (a server, a
 * benchmark with warm-up rounds): create binds the graph, allocates the two batches'
 * device memory, validates and schedules (and autotunes if asked); every run continues
 * for up to 'rounds' more rounds from the current state (genes, mean vector, global best)
 * and reports that call's rounds (round_time is measured from the start of the call);
 * p->eq0/el0/l0 seed the population at create; p->rounds is ignored. */
typedef struct deco_solver deco_solver;
deco_status deco_solver_create(deco_solver **out, const deco_graph *g, const deco_solve_params *p,
                               void *stream);
deco_status deco_solver_run(deco_solver *s, int32_t rounds, double *best_cut, uint8_t *best_z,
                            double *round_time, double *round_best, deco_solve_report *report);
/* Replace the early-stop targets (host [G]; NULL clears them). */
deco_status deco_solver_set_target(deco_solver *s, const double *target_cut);
void deco_solver_destroy(deco_solver *s);

/* ---------------------------------------------------------------------------------
 * Learned starting magnitudes (an extension; the paper's method is training-free): a
 * 3-layer message-passing network over [d_v/dbar, m_v/dbar, log(1+d_v) - log(1+dbar)]
 * (d = degree, m = mean neighbour degree, dbar = the graph's mean degree), hidden width
 * 64, h <- relu(h Ws + mean_nbr(h) Wn + b), output y = sigmoid(h wo + bo) in (0, 1). The
 * forward pass uses the parameters rounded to bfloat16 with float32 accumulation. The
 * parameters are one packed device float32 vector of deco_mpnn_num_params() values in the
 * order Ws1 (3x64), Wn1 (3x64), b1, Ws2 (64x64), Wn2, b2, Ws3, Wn3, b3, wo (64), bo (1);
 * matrices row-major [input][output]. Training minimises mean_v (y_v - t_v)^2 against
 * t_v = cut fraction of v's weight at a best vector (deco_mpnn_labels). All buffers are
 * device memory owned by the caller; the workspace holds activations for the backward pass.
 * --------------------------------------------------------------------------------- */
int32_t deco_mpnn_num_params(void);
deco_status deco_mpnn_workspace_size(const deco_graph *g, size_t *bytes);
/* y[n] = network output per node. Asynchronous. */
deco_status deco_mpnn_forward(const deco_graph *g, const float *params, float *y, void *workspace,
                              size_t workspace_bytes, void *stream);
/* For callers that cannot allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same forward pass with its activations in a
 * library-owned scratch array instead of a caller workspace. The scratch is a 32 MiB static
 * device array, one copy per GPU, held until the process ends (1,056 bytes per node: n <=
 * 31,774, else DECO_E_UNSUPPORTED before anything is launched). The call allocates nothing.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (several
 * streams or host threads) race and must be serialised by the caller. Asynchronous; y[n]
 * (device) as deco_mpnn_forward. */
deco_status deco_mpnn_forward_static(const deco_graph *g, const float *params, float *y, void *stream);
/* Loss (host double, after a synchronisation) and its gradient with respect to the
 * bfloat16-rounded parameters (device float32, same packing). */
deco_status deco_mpnn_loss_grad(const deco_graph *g, const float *params, const float *target,
                                float *grads, double *loss, void *workspace, size_t workspace_bytes,
                                void *stream);
/* One Adam step (Kingma and Ba; beta1 0.9, beta2 0.999, eps 1e-8) on the float32 masters;
 * m, v: device moment buffers of the same size, zero before step 1. */
deco_status deco_mpnn_adam(float *params, const float *grads, float *m, float *v, int32_t step, float lr,
                           void *stream);
/* t[v] = sum_u w_vu 1{z_u != z_v} / d_w(v) for a cut vector z (device bytes), 0 if isolated. */
deco_status deco_mpnn_labels(const deco_graph *g, const uint8_t *z, float *target, void *stream);

/* Host utility: one evolution step of Sec. 4.3 for the genome (eq, el, l). Members are
 * ranked by fitness (descending; ties to the lower index); the top half is kept in rank
 * order; ranked member K/2+j becomes member j perturbed by e' = clip(e + 0.2 N(0,1),
 * lo, hi) for each exponent and l' = clip(l + U{-1,0,1}, 1, lmax). Draws use the
 * generator above with counter (round, member, 6, 0/1). Host memory in and out. */
deco_status deco_evo_next(int32_t K, const double *fitness, const double *eq, const double *el,
                          const int32_t *l, double lo, double hi, int32_t lmax, uint64_t seed,
                          uint32_t round, double *eq_out, double *el_out, int32_t *l_out);

/* Initial population of the evolution-based search (Sec. 4.3: every member's combination is
 * drawn from the bounds). Member k (host arrays [K] out):
 *   eq[k], el[k] = lo + (hi - lo) u, u = (r >> 8) 2^-24 of words 0 and 1 of Philox counter
 *     (0xFFFFFFFF, k, 6, 6): the log10 step sizes of the unlifted and the lifted batch,
 *     uniform on [lo, hi);
 *   l[k] = 1 + (word 2 of that draw) mod lmax: the lift dimension, uniform on {1..lmax};
 *   Tq[k] = Tq_lo + (word 0 of counter (0xFFFFFFFF, k, 6, 3)) mod (Tq_hi - Tq_lo + 1), and
 *   Tl[k] likewise from counter (0xFFFFFFFF, k, 6, 5): the step counts, uniform on their
 *     ranges (relative bias of the modulo below 2^-19 for ranges up to 8192 counts).
 * deco_solver_create draws its population with this function (lo = -4, hi = -1, the bounds
 * of Sec. 5; counts from [T_min, T_q] and [T_l_min, T_l] when searched). DECO_E_INVAL for
 * K < 1, lmax < 1, !(lo <= hi), empty count ranges or NULL outputs. */
deco_status deco_evo_init(int32_t K, double lo, double hi, int32_t lmax, int32_t Tq_lo, int32_t Tq_hi,
                          int32_t Tl_lo, int32_t Tl_hi, uint64_t seed, double *eq, double *el, int32_t *l,
                          int32_t *Tq, int32_t *Tl);

/* Step counts after one evolution round (Sec. 4.3, the step-count half of the search): the
 * members are ranked as by deco_evo_next (descending fitness, ties to the lower index); the
 * top half keeps its counts in rank order and slot K/2 + j takes ranked member j's count
 * T0 as T' = floor(T0 (1 + 0.2 (2 eps' - 1))), eps' ~ U(0,1) (Philox counter (round, slot,
 * 6, 2 + 2 gene); gene 0: unlifted count, 1: lifted count), clipped to [T_lo, T_hi]. Host
 * arrays [K]. DECO_E_INVAL for K < 1, bad bounds or gene > 1. */
deco_status deco_evo_next_steps(int32_t K, const double *fitness, const int32_t *T, int32_t T_lo,
                                int32_t T_hi, uint64_t seed, uint32_t round, uint32_t gene,
                                int32_t *T_out);

/* Host utility: Philox4x32-10 of one counter/key (for known-answer tests). */
void deco_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Device check of the generator: out[i*4 + j] = Philox(ctr_i, key)[j] for
 * ctr_i = (i, c1, c2, c3), i < count (device uint32 out[count*4]). Asynchronous. */
deco_status deco_philox_device(uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed,
                               int32_t count, uint32_t *out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DECO_H */
