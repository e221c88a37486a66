/*
 * mc3.h -- C ABI of the MI355X many-configuration Markov-chain Monte Carlo (MCMCMC)
 * hot path for the Sherrington-Kirkpatrick (SK) spin glass.
 *
 * Method (paper: "Many-Configuration Markov-Chain Monte Carlo"):
 *   - Target: P_eq(s) proportional to exp(-beta E(s)) with the SK energy
 *     E(s) = -scale * sum_{i<j} J_ij s_i s_j, s_i in {-1,+1}
 *     (Sec. "The Sherrington-Kirkpatrick model"; the paper's +1/sqrt(L) sum J S S
 *     with unit-variance J is the same law with J -> -J/sqrt(L)).
 *   - Each step every chain generates a graph of configurations from its current
 *     state and moves to one node of it, drawn with
 *     P_node(c|T) = P_eq(c) P_gen(T|c) / sum_{c' in T} P_eq(c') P_gen(T|c')
 *     (App. "Markov chain of graphs of configurations", Eq.
 *     eq_det_balance_graph_solution with the normalisation of
 *     Eq. eq_normalization_p_c_T).
 *   - Graph: a tree on M+1 nodes populated from the position r of the current state
 *     (App. "General graph populating process"): by default the M-ary star (hub =
 *     node 0, leaves 1..M) with r drawn uniformly; breadth-first a-ary trees, the
 *     line-graph addition process and caller-given root laws are chosen by arity and
 *     law (mc3_graph_law).  Each edge e carries a flip set F_e of k_e ~ U{kmin..kmax}
 *     distinct sites that does not depend on the state, so the two-body law is
 *     symmetric: with a uniform root the tree is self-thermalising,
 *     P_node(v) = exp(-beta E_v) / sum_v' exp(-beta E_v'); other root laws add their
 *     log P_gen(T|c_v) to the exponents.
 *   - The set variant's generation and subset-visit probabilities (App. "Markov chain
 *     of sets of configurations") are a separate, context-free call
 *     (mc3_set_generation).
 *   - Rule METROPOLIS (M = 1): the single-update Metropolis rate min(1, e^{-beta dE})
 *     of Sec. "Problem statement", the paper's baseline.
 *
 * Conventions
 *   - Spin bitsets passed through this ABI: bit i of word i/32 set <=> s_i = -1 (the
 *     device keeps its own bit order inside each word).
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key (seed lo, seed hi)
 *     and counter (block, edge, step, tag<<28 | global chain).  Tags: 1 init,
 *     2 root, 3 edge, 4 select.  randint(w, n) = (w * n) >> 32.
 *   - All calls are asynchronous on the stream given at create time unless stated.
 *   - Results depend only on (config, couplings, seed, step numbers), never on the
 *     launch geometry.
 *
 * Errors: every call returns an mc3_status; no C++ exception crosses the ABI.  A
 * device error seen by a synchronising call (mc3_sync, mc3_measure, mc3_read_*)
 * poisons the context: later calls return MC3_E_STATE.  mc3_last_error gives text.
 */
#ifndef MC3_H
#define MC3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MC3_OK = 0,
    MC3_E_ARG = -1,         /* invalid argument or configuration */
    MC3_E_DEVICE = -3,      /* a HIP call or kernel failed */
    MC3_E_STATE = -4,       /* call out of order, or context poisoned */
    MC3_E_UNSUPPORTED = -5, /* valid request the library does not implement */
    MC3_E_NUMERIC = -6,     /* non-finite or inconsistent couplings */
    MC3_E_WORKSPACE = -7    /* workspace missing, too small or misaligned */
} mc3_status;

typedef enum {
    MC3_FP64 = 0,        /* scoring in FP64 on the FP64 matrix cores */
    MC3_SPLIT_BF16 = 1   /* J = hi + mid + lo (three BF16 terms), spins exact in BF16,
                            FP32 accumulation on the BF16 matrix cores, FP64 epilogue */
} mc3_precision;

typedef enum {
    MC3_RULE_MCMCMC = 0,     /* node rule over the M+1 nodes of the graph */
    MC3_RULE_METROPOLIS = 1  /* single proposal, Metropolis rate; requires M == 1 */
} mc3_rule;

/* How node energies are obtained.
 *   GEMM:  every candidate's energy from the dense pair sum, J.S on the matrix cores
 *          (precision as configured); any flip-set size.
 *   DELTA: energies as differences from the current state, in FP64: the device keeps
 *          U = sum_{i<j} J_ij s_i s_j and the local field h = J s per chain, and node v
 *          differs from the current node by the path flip set D = F_r xor F_v, so
 *          dU = -2 sum_{i in D} s_i h_i + 4 sum_{i<j in D} J_ij s_i s_j (|D| + |D|^2/2
 *          couplings per candidate instead of N^2); a move updates h with the |D|
 *          rows of J.  All steps of a chain run in one persistent workgroup, every
 *          chain of every instance of a batch in one launch.  Limits: either (small
 *          flip sets, any tree) kmax <= 16, M <= 512, N <= 4096, kmax times the
 *          longest path between two nodes (in edges) <= 32 and the per-chain state
 *          within 64 KiB of LDS; or (the star, flip sets of any size) the per-chain
 *          state within 160 KiB of LDS: 16 N + 24 (M+1) + 8 W + 4 M W + 8 kmax bytes
 *          for the batch's largest N, M, kmax and W = 4 ceil(N/128)
 *          (MC3_E_UNSUPPORTED otherwise); only mc3_step_n moves the chains
 *          (mc3_propose, mc3_score_candidates, mc3_select, mc3_read_candidates and
 *          mc3_step_n_per_instance return MC3_E_UNSUPPORTED).  `precision` is unused.
 *   AUTO:  DELTA where its limits hold and kmax times the longest path is at most
 *          16, else GEMM. */
/* How the current state is placed in the graph (the root law of the populating
 * process).  The graph is the tree on M+1 nodes labelled breadth first with the
 * parent of node v >= 1 at (v-1)/arity; edge v joins node v to its parent and carries
 * the flip set F_v; node v holds the state at node 0 with the flip sets of the edges
 * from node 0 down to v flipped (the current state sits at the root position r).
 *   UNIFORM: r ~ U{0..M}, the populating process with a uniform root (App. "General
 *            graph populating process"): self-thermalising, node weights
 *            exp(-beta E_v).  arity = M is the M-ary star; the paper's SK trees are
 *            arities 2, 3, 16 with 127, 121, 273 nodes (Fig. fig_sk).
 *   LINE:    the line-graph addition process (App. "Line-graph addition process";
 *            requires arity 1): M nodes added one by one at either end with
 *            probability 1/2, so r ~ Binomial(M, 1/2) (bit j of the root stream's
 *            words sends addition j left) and P_gen(T|c_v) carries C(M, v) / 2^M
 *            (the reading of the garbled prefactor); node weights
 *            exp(-beta E_v) C(M, v), applied as the log-prior
 *            lgamma(M+1) - lgamma(v+1) - lgamma(M-v+1).
 *   TABLE:   a root law given by the caller (App. "General graph populating
 *            process": the root distribution p_r of a tree is free), any arity: weights
 *            g_0..g_M >= 0 per instance (law_table), taken in fixed point as
 *            q_v = floor(g_v / S * 2^52), S = sum of g in node order; the root is
 *            r = min { v : q_0 + .. + q_v > t }, t = floor(u53 W / 2^53) with u53 from
 *            root-stream words 0 and 1 and W = sum q.  With flip sets that do not
 *            depend on the state P_gen(T|c_v) is p_v times a factor common to the
 *            nodes, so node weights are exp(-beta E_v) q_v (log-prior log q_v; q_v = 0:
 *            never the root, never chosen).  The three-configuration process with a
 *            general p (Sec. "Generalization to three configurations per Monte Carlo
 *            step") is arity 1, M = 2, weights (q/2, p, q/2), q = 1 - p; the line-graph
 *            addition process with probability p of adding at node 0's end is arity 1
 *            with weights C(M, v) p^v q^(M-v).
 *   BIASED:  a two-body proposal that depends on the state (Sec. "Problem statement"
 *            allows any ergodic proposal): on the star (arity 0 or >= M) with
 *            single-site edges (kmin = kmax = 1) and a uniform root, the site of an
 *            edge is drawn from the state it is generated from with probability
 *            proportional to exp(-bias dE_i), dE_i = 2 scale s_i h_i the energy change
 *            of flipping site i (fixed point: q_i = floor(exp(a_i - max a) 2^52),
 *            a_i = -(bias ((2 scale) (s_i h_i))), drawn with u53 of words 0, 1 of the
 *            edge's stream).  r = 0: the hub is the current state; r >= 1: the hub is
 *            the current state with site i_r ~ p(.|current) flipped; the other leaves
 *            flip sites ~ p(.|hub).  Node weights exp(-beta E_v) rho_v with
 *            rho_v = P_gen(T|c_v) / P_gen(T|hub) = p_{i_v}(c_v) / p_{i_v}(hub) (taken as
 *            (q_{i_v}(c_v) W(hub)) / (q_{i_v}(hub) W(c_v))), rho_hub = 1; if the hub
 *            cannot generate leaf r the chain stays.  Runs on the field-update scorer
 *            (scorer DELTA or AUTO; GEMM is MC3_E_ARG), N <= 1024, M <= 512
 *            (MC3_E_UNSUPPORTED beyond); rule MCMCMC.  These proposals depend on the
 *            state, so they are drawn within each step, never ahead. */
typedef enum {
    MC3_LAW_UNIFORM = 0,
    MC3_LAW_LINE = 1,
    MC3_LAW_TABLE = 2,
    MC3_LAW_BIASED = 3
} mc3_graph_law;

typedef enum {
    MC3_SCORER_GEMM = 0,
    MC3_SCORER_DELTA = 1,
    MC3_SCORER_AUTO = 2
} mc3_scorer;

/* How the pair-sum scorers carry each chain's energy from step to step (the field-
 * update scorer always carries exact FP64 differences).  The carried quantity is the
 * unscaled pair sum U = sum_{i<j} J_ij s_i s_j in FP64, E = -(scale U).
 *   EXACT:  on a move, U += dU(D*) computed in FP64 from the |D*| rows of J, D* the set
 *           of sites where the new state differs from the old one:
 *           dU = -2 sum_{i in D*} s_i sum_{j not in D*} J_ij s_j (old spins); exact
 *           integers for +-1 couplings.  Costs |D*| N coupling reads per move.
 *           Inside a run of steps each move's difference is added by the next
 *           step's selection; every call that selects (mc3_select, mc3_select_betas,
 *           the mc3_step_n family) returns with the carried energies and the records
 *           complete.
 *   SCORED: U = the chosen candidate's pair sum as scored (split BF16 on the split
 *           path), no extra reads. */
typedef enum {
    MC3_ENERGY_EXACT = 0,
    MC3_ENERGY_SCORED = 1
} mc3_energy_update;

/* Kinds of seeded couplings (mc3_generate_couplings). */
typedef enum {
    MC3_J_PM1 = 0,
    MC3_J_GAUSS = 1
} mc3_coupling;

/* One SK instance and its chains.  Constraints: 2 <= N <= 8192, 1 <= M <= 4000,
 * 1 <= chains, 1 <= kmin <= kmax <= N, chains * M <= 2^24, rule METROPOLIS => M == 1. */
typedef struct {
    int32_t N;               /* spins */
    int32_t M;               /* graph size minus one: leaves of the star = new configurations per chain-step */
    int32_t chains;          /* independent chains */
    int32_t kmin, kmax;      /* flip-set size range of every edge */
    int32_t precision;       /* mc3_precision */
    int32_t rule;            /* mc3_rule */
    int32_t trace_steps;     /* capacity of the per-step record ring (>= 0) */
    uint64_t seed;           /* Philox key */
    uint32_t chain_base;     /* global index of chain 0 in the Philox counter */
    int32_t mean_steps;      /* capacity of the per-step chain-mean trace ring (>= 0) */
    double near_tie_tol;     /* selection margin below which a step is flagged (a fixed threshold);
                                < 0 => the default 4 beta eps_E per step, eps_E = N 2^-24 for
                                split-BF16 scores and N 2^-40 for FP64 scores (the largest change
                                of an energy's rounding, see mc3_select) */
    int32_t scorer;          /* mc3_scorer */
    int32_t arity;           /* graph tree arity; 0 or >= M: the M-ary star */
    int32_t law;             /* mc3_graph_law */
    const double* law_table; /* law TABLE: host [M+1] root weights, copied by mc3_create;
                                otherwise ignored */
    int32_t tile_cols;       /* split-BF16 scoring tile width (columns per work unit): 0 = by
                                the instance's column count (512 from 2048 columns up, 128 up
                                to 128, 256 between); 128, 256 or 512 = that width.  Results
                                do not depend on it.  Ignored by the FP64 and field-update
                                scorers; any other value is MC3_E_ARG */
    int32_t recompute_every; /* K > 0: after the selection of every global step t with
                                (t + 1) % K == 0 every chain's energy is recomputed in FP64
                                from its spins (as mc3_recompute); 0: only mc3_recompute */
    int32_t energy_update;   /* an mc3_energy_update value, for the pair-sum scorers */
    double drift_tol;        /* a recompute whose |E_carried - E_recomputed| exceeds
                                drift_tol (|E_recomputed| + 1) counts as a drift event;
                                < 0 => 1e-9 */
    double bias;             /* law BIASED: the proposal's bias (alpha); otherwise ignored */
} mc3_config;

/* One instance of a batch: its size, graph size, chains and flip-set range, with the
 * constraints of mc3_config. */
typedef struct {
    int32_t N, M, chains, kmin, kmax;
} mc3_instance_desc;

/* A batch of independent SK instances sharing precision, rule, seed and ring sizes
 * (many small instances in one set of launches).  The chains of all instances are
 * numbered consecutively in instance order ("global chains"): global chain g uses
 * Philox chain index chain_base + g, so instance i with first global chain g_i runs
 * exactly as a single-instance context with chain_base + g_i would. */
typedef struct {
    int32_t n_instances;     /* 1 .. 2^20 */
    int32_t precision;       /* mc3_precision */
    int32_t rule;            /* mc3_rule */
    int32_t trace_steps;     /* record ring capacity (steps), records of all global chains */
    int32_t mean_steps;      /* chain-mean trace capacity (means over all global chains) */
    uint32_t chain_base;     /* Philox chain index of global chain 0 */
    uint64_t seed;           /* Philox key */
    double near_tie_tol;     /* < 0 => default */
    const mc3_instance_desc* instances;  /* [n_instances], copied by mc3_batch_create */
    int32_t scorer;          /* mc3_scorer */
    int32_t arity;           /* graph tree arity of every instance; 0 or >= M: the star */
    int32_t law;             /* mc3_graph_law */
    const double* law_table; /* law TABLE: host root weights of every instance, instance i's
                                M_i+1 values after those of instances 0..i-1; copied by
                                mc3_batch_create; otherwise ignored */
    int32_t tile_cols;       /* split-BF16 scoring tile width of every instance, as in
                                mc3_config */
    int32_t recompute_every; /* as in mc3_config */
    int32_t energy_update;   /* as in mc3_config */
    double drift_tol;        /* as in mc3_config */
    double bias;             /* as in mc3_config */
} mc3_batch_config;

/* Per-step, per-chain record (40 bytes). */
typedef struct {
    int32_t r;          /* position of the state the graph was generated from (root) */
    int32_t vstar;      /* selected node; METROPOLIS: 1 = accepted, 0 = rejected */
    double e_cur;       /* carried energy of the state after the step (-(scale U)) */
    double e_bar;       /* node-weighted energy sum_v P_node(v) E_v (Eq. eq_monte_carlo_graph);
                           METROPOLIS: e_cur */
    double margin;      /* distance of the draw to the edges of the selected interval,
                           as a fraction of the total weight (METROPOLIS: |u - rate|) */
    uint32_t flags;     /* bit 0: near tie (margin below the step's threshold); bit 1: moved */
    uint32_t step;      /* global step number */
} mc3_record;

/* Aggregate counters since the last mc3_init_chains. */
typedef struct {
    int64_t steps_done;    /* chain-steps summed over chains / chains */
    int64_t moves;         /* chain-steps that changed the state */
    int64_t near_ties;     /* chain-steps flagged as near ties */
    double min_margin;     /* smallest selection margin seen */
    double max_drift;      /* largest |E_carried - E_recomputed| at a recompute */
    int64_t recomputes;    /* recomputes (periodic and mc3_recompute) */
    int64_t drift_events;  /* chain recomputes whose drift exceeded the drift tolerance */
} mc3_summary;

/* A linear inverse-temperature schedule: step t has
 * beta0 + (beta1 - beta0) (t / (total - 1)), beta0 if total <= 1. */
typedef struct {
    double beta0, beta1;
    int64_t total;
} mc3_schedule;

typedef struct mc3_ctx mc3_ctx;

/* Device workspace (bytes) the context needs for this configuration.  The caller
 * allocates it (any device allocator; 256-byte aligned) and lends it to mc3_create. */
mc3_status mc3_workspace_size(const mc3_config* cfg, size_t* bytes);

/* Create a context on the current HIP device.  `workspace` is a device pointer of at
 * least mc3_workspace_size bytes, borrowed for the lifetime of the context; `stream`
 * is a hipStream_t (NULL = default stream), borrowed likewise; every kernel of the
 * context runs on it.  Performs no device memory allocation and creates no stream
 * (mc3_step_n_graph later creates one to capture on).
 * Validates the configuration before any HIP call. */
mc3_status mc3_create(const mc3_config* cfg, void* workspace, size_t bytes, void* stream, mc3_ctx** out);

/* Largest workspace a context from mc3_create_noalloc can have: 16 MiB. */
#define MC3_NOALLOC_BYTES (16u << 20)

/* mc3_create for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the workspace is a
 * fixed array of MC3_NOALLOC_BYTES in the library's device code, one per GPU, held
 * until the process ends; no hipMalloc, hipFree or other allocating call is made.
 * Every other call works on the context as on one from mc3_create.  The array is
 * shared by every context of this kind on a device: one such context per device at a
 * time (MC3_E_STATE while another one lives; mc3_destroy waits for its stream and
 * frees the array for the next).  Calls from several threads that overlap on one
 * device's array race.  The array keeps what the last context left in it; the calls
 * that set a context up (mc3_init_couplings, mc3_init_chains, mc3_checkpoint_load)
 * clear or write everything a step reads first, as they do for a fresh workspace.
 * Errors: MC3_E_ARG / MC3_E_UNSUPPORTED as mc3_create; MC3_E_WORKSPACE when
 * mc3_workspace_size(cfg) exceeds MC3_NOALLOC_BYTES; MC3_E_DEVICE when the array's
 * address cannot be obtained. */
mc3_status mc3_create_noalloc(const mc3_config* cfg, void* stream, mc3_ctx** out);

/* Batch forms of mc3_workspace_size and mc3_create (same contracts).  Every call
 * below works on a batch context: per-chain arrays span the global chains, the
 * energies of mc3_score_candidates are the instances' [chains][M] blocks one after
 * another, and spins passed to mc3_init_chains are the instances' [chains][N] blocks
 * one after another.  A single-instance context is a batch of one. */
mc3_status mc3_batch_workspace_size(const mc3_batch_config* cfg, size_t* bytes);
mc3_status mc3_batch_create(const mc3_batch_config* cfg, void* workspace, size_t bytes, void* stream,
                            mc3_ctx** out);

/* Release the host-side context (the workspace stays the caller's). */
mc3_status mc3_destroy(mc3_ctx* ctx);

/* Load couplings: J is a host array of N*N doubles, row-major with leading dimension
 * ld >= N; only the strict upper triangle i<j is read (J is taken as symmetric with
 * zero diagonal: the device mirrors the upper triangle below the diagonal and clears
 * the diagonal, so whatever the array holds at or below the diagonal, NaN included,
 * is ignored by every scorer).  Energies are E = -scale * sum_{i<j} J_ij s_i s_j.
 * Values i<j must be finite (MC3_E_NUMERIC otherwise).  The array is copied before return
 * (synchronous on the stream); the device keeps J in FP64 and, for the split
 * precision, as three BF16 terms hi = bf16(J), mid = bf16(J - hi),
 * lo = bf16(J - hi - mid), each packed in matrix-core fragment order. */
mc3_status mc3_init_couplings(mc3_ctx* ctx, const double* J, int64_t ld, double scale);

/* Seeded SK instances generated on the device, in place of mc3_init_couplings for
 * instance `instance` (0 for a single-instance context).  The paper's SK couplings
 * are Gaussian (Sec. "The Sherrington-Kirkpatrick model"); the +-1 kind has integer
 * energies, so trajectories can be compared bit for bit.  Pair i < j reads block j
 * of the coupling stream (Philox4x32-10, key = seed, counter = (j, i, 0, 5 << 28)),
 * words w0..w3:
 *   MC3_J_PM1:   J_ij = +1 if bit 0 of w0 is set, else -1; energy scale 1/sqrt(N).
 *   MC3_J_GAUSS: Box-Muller, u1 = (u53(w0, w1) + 1) / 2^53, u2 = u53(w2, w3) / 2^53,
 *                J_ij = (sqrt(-2 ln u1) cos(2 pi u2)) * (1/sqrt(N)); energy scale 1
 *                (device log and cos: within an ulp or two of any other libm).
 * J is symmetric with a zero diagonal.  Synchronises like mc3_init_couplings.  Errors:
 * MC3_E_ARG for an unknown kind or instance. */
mc3_status mc3_generate_couplings(mc3_ctx* ctx, int32_t instance, int32_t kind, uint64_t seed);

/* mc3_init_couplings for instance `instance` of a batch (mc3_init_couplings loads
 * instance 0).  Every instance needs its couplings before mc3_init_chains. */
mc3_status mc3_init_couplings_instance(mc3_ctx* ctx, int32_t instance, const double* J, int64_t ld,
                                       double scale);

/* Set the chains' states: spins is a host array [chains][N] of +-1 (int8), or NULL to
 * draw them from the init stream (bit i%32 of word i/32 of stream (tag 1, chain,
 * step 0, edge 0); set bit = spin -1).  Computes each chain's FP64 energy and clears
 * the record ring and the summary.  Requires couplings. */
mc3_status mc3_init_chains(mc3_ctx* ctx, const int8_t* spins);

/* Draw the graph of every chain at global step `step` (App. "General graph
 * populating process", uniform root): root r = randint(word 0 of (tag 2), M+1)
 * (METROPOLIS: r = 0); for each edge e = 1..M of stream (tag 3, edge e):
 * k_e = kmin + randint(word 0, kmax-kmin+1), then Floyd's k-of-N on words 1..k_e.
 * Node configurations: r = 0: hub = s, leaf e = s^F_e; r >= 1: leaf r = s,
 * hub = s^F_r, leaf e = s^F_r^F_e.  The M non-current nodes of chain c are its
 * candidate columns c*M + m, m = 0..M-1: column m is leaf m+1, except that for a
 * root r >= 1 column r-1 is the hub.  Stores the flip sets, the roots and, per chain,
 * base = s^F_r; candidates are formed from these inside the scoring kernels. */
mc3_status mc3_propose(mc3_ctx* ctx, uint32_t step);

/* Score the candidates of the last mc3_propose: E(c) = -scale sum_{i<j} J_ij c_i c_j
 * for every candidate column, on the matrix cores (Sec. "The Sherrington-Kirkpatrick
 * model").  If E_out is not NULL it receives the energies, a device array
 * [chains][M] of doubles owned by the caller. */
mc3_status mc3_score_candidates(mc3_ctx* ctx, double* E_out);

/* Apply the node rule to the scored graphs at step `step` with inverse temperature
 * beta and move every chain (App. "Markov chain of graphs of configurations"):
 * Emin = min_v E_v (the current node's E is its carried energy);
 * w_v = exp(-(beta (E_v - Emin))) in FP64; q_v = floor(w_v 2^52) (exact integers);
 * Q_v their inclusive prefix sum in node order 0..M, W = Q_M;
 * t = floor(u53 W / 2^53) with u53 from words 0,1 of (tag 4);
 * v* = min{v : Q_v > t}.  METROPOLIS: accept iff dE <= 0 or u53/2^53 < exp(-(beta dE)).
 * The carried energy then follows the configuration's energy_update.  The margin (the
 * draw's distance to the edges of its interval, as a fraction of W) is flagged as a
 * near tie below the threshold: errors of at most eps_E in every node energy move
 * each interval edge by at most beta eps_E of W, so an unflagged draw picks the node
 * exact arithmetic would.  Writes one mc3_record per chain into the ring (slot
 * step % trace_steps); with recompute_every = K and (step + 1) % K == 0 the periodic
 * recompute follows. */
mc3_status mc3_select(mc3_ctx* ctx, uint32_t step, double beta);

/* mc3_select with an inverse temperature per instance: beta is a host array
 * [n_instances] (copied; the call waits for the stream before taking it). */
mc3_status mc3_select_betas(mc3_ctx* ctx, uint32_t step, const double* beta);

/* n steps starting at global step step0: propose, score, select each step, with
 * beta_t = beta0 + (beta1 - beta0) * (t / (total - 1)) for t = step0 .. step0+n-1
 * (beta0 if total <= 1).  Flip sets and roots do not depend on the states, so the
 * proposals of up to 16 steps are drawn in one launch into a ring in the workspace;
 * the results are those of the step-by-step calls. */
mc3_status mc3_step_n(mc3_ctx* ctx, uint32_t step0, int64_t n, double beta0, double beta1, int64_t total);

/* mc3_step_n with a schedule per instance: sched is a host array [n_instances] (copied;
 * the call waits for the stream before taking it); instance i's chains take beta_t of
 * sched[i].  MC3_E_ARG for a negative or non-finite beta or a total outside
 * [0, 2^53]. */
mc3_status mc3_step_n_schedules(mc3_ctx* ctx, uint32_t step0, int64_t n, const mc3_schedule* sched);

/* The steps of mc3_step_n (same arguments, same results bit for bit), replayed from a
 * HIP graph: the launches of L steps (L a multiple of the proposal group of up to 16
 * steps, of the proposal ring's length and of 2, at most 272) are captured once on a
 * stream of the context's own and replayed on the context's stream; a step counter in
 * the workspace gives the replayed proposal, selection and means kernels their step,
 * and the selection forms beta_t from (beta0, beta1, total) on the device in the
 * host's operation order.  The capture is kept for later calls with the same schedule
 * and the same step0 modulo L.  Runs of fewer than L + 16 steps, and the last 16 to
 * L + 15 steps of a run, are launched as in mc3_step_n; with the field-update scorer
 * or a periodic recompute (recompute_every > 0) this is mc3_step_n.  Scoring launches inside replays are not timed
 * (mc3_timing_enable).  For step loops whose launches, not their kernels, take the
 * time (small N and M). */
mc3_status mc3_step_n_graph(mc3_ctx* ctx, uint32_t step0, int64_t n, double beta0, double beta1, int64_t total);

/* The steps of mc3_step_n, launched instance by instance (propose, score and select
 * of instance 0, then of instance 1, ...) on the context's stream, without the
 * overlap of proposal and scoring.  Same results as mc3_step_n; it is the cost of
 * running the instances one at a time, against which the batched launches are
 * measured. */
mc3_status mc3_step_n_per_instance(mc3_ctx* ctx, uint32_t step0, int64_t n, double beta0, double beta1,
                                   int64_t total);

/* Recompute every chain's energy from its spins in FP64 on the matrix cores
 * (U = (1/2) sum_i s_i (J s)_i, the symmetric zero-diagonal J), record
 * |E_carried - E_recomputed| (its largest value per chain, and a drift event when it
 * exceeds drift_tol (|E| + 1)) in the summary, and carry the recomputed value (the
 * repair).  Synchronises. */
mc3_status mc3_recompute(mc3_ctx* ctx);

/* Synchronise; copy the chains' energies (host [chains], may be NULL), spins (host
 * bitsets [chains][ceil(N/32)] uint32, may be NULL) and the summary (may be NULL).
 * In a batch: [global chains], and the bitset row length is ceil(max N / 32) words
 * (zero beyond each instance's own). */
mc3_status mc3_measure(mc3_ctx* ctx, double* e_cur, uint32_t* spin_bits, mc3_summary* summary);

/* Synchronise and copy `n` steps of records starting at global step `first`
 * (they must still be in the ring) into host [n][chains]. */
mc3_status mc3_read_records(mc3_ctx* ctx, uint32_t first, int32_t n, mc3_record* out);

/* Synchronise and copy the candidate bitsets of the last mc3_propose into host
 * [chains][M][ceil(N/32)] uint32, and the roots into host [chains] (either may be NULL).
 * Single-instance contexts only (MC3_E_UNSUPPORTED for a batch of several). */
mc3_status mc3_read_candidates(mc3_ctx* ctx, uint32_t* bits, int32_t* roots);

/* Synchronise and copy the chain means of steps first .. first+n-1 (still in the
 * trace ring of capacity mean_steps) into host [n][2]: {mean over chains of the
 * current energy after the step, mean of the node-weighted energy of the step's graph
 * (Eq. eq_monte_carlo_graph)}.  Both means are fixed-order device reductions. */
mc3_status mc3_read_means(mc3_ctx* ctx, uint32_t first, int32_t n, double* out);

/* Measurement aid.  on = 0 disables; on = k >= 1 brackets every k-th scoring-kernel
 * launch (mc3_score_candidates, mc3_step_n; the first one after enabling, then every
 * k-th) with timestamp-only HIP events (no system-scope cache flush) recorded on the
 * stream it runs on: k = 1 times every launch, a larger k keeps the events' own cost
 * (a few microseconds per record) out of a long run.  Enabling resets the totals.
 * MC3_E_ARG for on < 0. */
mc3_status mc3_timing_enable(mc3_ctx* ctx, int32_t on);

/* Synchronise; total milliseconds of the timed scoring launches and their number. */
mc3_status mc3_timing_read(mc3_ctx* ctx, double* total_ms, int64_t* launches);

/* Checkpoint of the chains: spins, carried energies (field-update scorer: also the pair
 * sums and fields), counters and steps done, as a self-describing host buffer (header,
 * instance shapes, arrays; the record and means rings are not included).  With
 * buf == NULL, *bytes receives the size needed; otherwise *bytes is the buffer's size
 * on entry and the size written on return.  Synchronises.  For resuming a run after
 * the process that made it ended. */
mc3_status mc3_checkpoint_save(mc3_ctx* ctx, void* buf, size_t* bytes);

/* Restore a checkpoint into a context of the same batch shape (instances, N, M,
 * chains) and scorer, after mc3_init_couplings of every instance, in place of
 * mc3_init_chains (the rings are cleared).  The steps that follow equal, bit for
 * bit, those the saving context would have run with the same step numbers.
 * MC3_E_ARG for a buffer of another shape or not a checkpoint. */
mc3_status mc3_checkpoint_load(mc3_ctx* ctx, const void* buf, size_t bytes);

/* Wait for the stream; report any device error. */
mc3_status mc3_sync(mc3_ctx* ctx);

/* Text of the last error on this context ("" if none); valid until the next call. */
const char* mc3_last_error(const mc3_ctx* ctx);

/* The set variant (App. "Markov chain of sets of configurations"): generation
 * probabilities of a set from its subsets and the probabilities of visiting each
 * subset, for n_sets sets of n elements at once; needs no context.
 * A set S = {0..n-1} grows from a nonempty subset X by additions (Sec. "Stochastic
 * generation of the set"): a parent chosen uniformly among the current elements
 * generates the new element e with probability G[e][parent]; S is reached when the
 * n - |X| additions bring exactly the elements of S \ X, in any order.
 *   G        device [n_sets][n][n] FP64, G[e][p] = P_gen(e | p) (row: new element).
 *   out      device [n_sets][2^n] FP64: out[X] = P_gen(S | X) for every bitmask X
 *            (out[S] = 1, out[0] = 0), from the recursion of Sec. "Recursive
 *            exponential formula for the generation probability" over subsets of
 *            decreasing size, out[X] = (1/|X|) sum_{e not in X} (sum_{p in X} G[e][p])
 *            out[X + e] (the prefactor fixed by the sum over insertion orders; the
 *            printed ones are garbled).
 *   peq      optional device [n_sets][2^n]: the equilibrium probabilities P_eq(X) of
 *            the proper subsets (entry S ignored; App. "Markov chain of sets of
 *            configurations": lambda_|X| w(X) / N_n); with it
 *   peq_set  device [n_sets]: P_eq(S) = sum_{X != S} P_eq(X) out[X] (Eq. eq_P_eq_n),
 *   psub     device [n_sets][2^n]: P_subset(X | S) = P_eq(X) out[X] / P_eq(S)
 *            (Eq. eq_p_S_S), psub[S] = 0; it sums to 1 over X.
 * Runs on `stream` (a hipStream_t, NULL = default) and returns without waiting.
 * MC3_E_ARG for 1 > n or n > 20, n_sets < 1, n_sets 2^n > 2^28, a NULL G or out, peq
 * without psub and peq_set (or the reverse), or a pointer that is not device memory;
 * MC3_E_DEVICE if a launch fails.  The caller owns every buffer. */
mc3_status mc3_set_generation(const double* G, int32_t n, int32_t n_sets, double* out, const double* peq,
                              double* psub, double* peq_set, void* stream);

/* Library version string. */
const char* mc3_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MC3_H */
