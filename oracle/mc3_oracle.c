/*
 * mc3_oracle.c -- plain, slow FP64 CPU oracle for many-configuration Markov-chain
 * Monte Carlo (MCMCMC) on the Sherrington-Kirkpatrick spin glass.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the GPU library is checked
 * against.  Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header, table or constant generator with the HIP
 * library; both were written separately from the same written definitions.
 *
 * What it follows (paper: "Many-Configuration Markov-Chain Monte Carlo"):
 *  - SK energy, Sec. "The Sherrington-Kirkpatrick model": a pair sum over j<k of
 *    couplings times spin products.  Convention used here (reading C1): the sign is
 *    folded into the coupling, E(s) = -scale * sum_{i<j} J_ij s_i s_j.
 *  - Markov chain of undirected graphs, App. "Markov chain of graphs of
 *    configurations": the next graph is generated from one node of the current
 *    graph, chosen with P_node(c|T) = P_eq(c) P_gen(T|c) / P_eq(T), normalised over
 *    the nodes of T (Eq. eq_det_balance_graph_solution with the normalisation
 *    Eq. eq_normalization_p_c_T).
 *  - Graph generation, App. "General graph populating process": a tree shape is
 *    fixed, the current state is placed at a root drawn uniformly, and every edge is
 *    populated with a two-body generation probability.  With a uniform root and a
 *    symmetric two-body law the tree is self-thermalising: P_gen(T|c_v) is the same
 *    for every node, so P_node reduces to exp(-beta E_v) normalised over the nodes.
 *    The trees used are labelled breadth first: node 0 on top, the parent of node
 *    v >= 1 is (v-1)/a for arity a, edge e joins node e to its parent and carries a
 *    flip set F_e.  Arity M is the star (hub 0, leaves 1..M); the paper's k-ary trees
 *    (Fig. fig_sk) are arities 2, 3 and 16.  Node v holds the current state with the
 *    flip sets of every edge on the path from the root position r to v flipped.
 *  - Line-graph addition process, App. "Line-graph addition process": starting from
 *    the current state, M nodes are added, each at the left or right end with
 *    probability 1/2.  With flip sets that do not depend on the state, this is the
 *    line (arity 1) with the current state at position r ~ Binomial(M, 1/2), and
 *    P_gen(T|c_v) carries the factor C(M, v) / 2^M (the printed prefactor is
 *    garbled; C(L-1, k) / 2^(L-1) with L = M+1 nodes is the reading taken), which
 *    enters the node rule as the log-prior log C(M, v).
 *  - A general root law, App. "General graph populating process" (the root
 *    distribution p_r is free; with a symmetric two-body law P_gen(T|c_v) is then
 *    p_v times a product common to all nodes): the caller gives weights g_v, the root
 *    is drawn from them in fixed point and the node rule carries log p_v.  The
 *    three-configuration process of Sec. "Generalization to three configurations per
 *    Monte Carlo step" with a general p is the line of three nodes with root weights
 *    (q/2, p, q/2), q = 1 - p, and the line-graph addition process with a bias p
 *    toward node 0 is the line with weights C(M, v) p^v q^(M-v).
 *  - A state-dependent two-body proposal (Sec. "Problem statement": any ergodic
 *    proposal; the paper's motivation for graphs includes biased proposals): single
 *    sites drawn with probability proportional to exp(-alpha dE_i) from the state the
 *    edge is generated from, on the star with a uniform root; the node rule carries
 *    P_gen(T|c_v) / P_gen(T|hub) (mc3o_biased_step).
 *  - Standard MCMC with the Metropolis rate min(1, ratio), Sec. "Problem statement",
 *    for the single-update baseline (rule METROPOLIS, M = 1).
 *  - Observables as node-weighted averages over the graph, Eq. eq_monte_carlo_graph.
 *  - The set variant's generation probability P_gen(S | X), Sec. "Stochastic
 *    generation of the set", summed over every order of the added elements.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), keyed by the seed; the counter names the
 * purpose of the draw (tag), the chain, the step, the edge and the block index.
 * Distinct k-subsets: R. W. Floyd's algorithm (Bentley & Floyd, CACM 30(9), 1987).
 * exp: Cody-Waite argument reduction by ln 2 and a degree-13 Taylor polynomial.
 *
 * Compile with -O2 -ffp-contract=off (no fused multiply-add anywhere).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ------------------------------------------------------------------ Philox4x32-10 */

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

/* One Philox4x32-10 block: 10 rounds of the S-box/permutation round of SC'11,
 * with the Weyl key schedule bumped between rounds. */
void mc3o_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Stream tags (counter word 3, top 4 bits). */
enum { TAG_INIT = 1, TAG_ROOT = 2, TAG_EDGE = 3, TAG_SELECT = 4 };

/* Word n of the stream (tag, chain, step, edge):
 * counter = (n / 4, edge, step, tag << 28 | chain), key = (seed lo, seed hi),
 * word = block[n % 4]. */
uint32_t mc3o_word(uint64_t seed, uint32_t tag, uint32_t chain, uint32_t step,
                   uint32_t edge, uint32_t n)
{
    uint32_t ctr[4] = { n / 4u, edge, step, (tag << 28) | (chain & 0x0FFFFFFFu) };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t out[4];
    mc3o_philox(ctr, key, out);
    return out[n % 4u];
}

/* Integer in [0, n) from one 32-bit word: floor(w * n / 2^32). */
uint32_t mc3o_randint(uint32_t w, uint32_t n)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

/* 53-bit uniform integer from two words: top 27 bits of w0, top 26 bits of w1. */
uint64_t mc3o_u53(uint32_t w0, uint32_t w1)
{
    return ((uint64_t)(w0 >> 5) << 26) | (uint64_t)(w1 >> 6);
}

/* Couplings of an SK instance from a seed (the instance generator; the paper draws
 * Gaussian couplings, Sec. "The Sherrington-Kirkpatrick model"; the +-1 kind gives
 * integer energies).  Pair a < b reads block b of the coupling stream (tag 5,
 * chain 0, step 0, edge a), words w0..w3.
 *   kind 0: J_ab = +1 if bit 0 of w0 is set, else -1 (energy scale 1/sqrt(N)).
 *   kind 1: Box-Muller, u1 = (u53(w0, w1) + 1) / 2^53 in (0, 1],
 *           u2 = u53(w2, w3) / 2^53 in [0, 1), z = sqrt(-2 ln u1) cos(2 pi u2),
 *           J_ab = z * (1 / sqrt(N)) (energy scale 1).
 * J is N x N row-major, symmetric, zero diagonal.  Returns 0, or -1 for a bad kind. */
int mc3o_couplings(int N, int kind, uint64_t seed, double* J)
{
    if (kind != 0 && kind != 1) return -1;
    const double inv_sqrt_n = 1.0 / sqrt((double)N);
    const double two_pi = 6.283185307179586;
    for (int a = 0; a < N; ++a) {
        J[(size_t)a * N + a] = 0.0;
        for (int b = a + 1; b < N; ++b) {
            uint32_t w[4];
            for (int q = 0; q < 4; ++q) w[q] = mc3o_word(seed, 5u, 0u, 0u, (uint32_t)a, 4u * (uint32_t)b + (uint32_t)q);
            double v;
            if (kind == 0) {
                v = (w[0] & 1u) ? 1.0 : -1.0;
            } else {
                const double u1 = ((double)mc3o_u53(w[0], w[1]) + 1.0) * 0x1.0p-53;
                const double u2 = (double)mc3o_u53(w[2], w[3]) * 0x1.0p-53;
                const double z = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
                v = z * inv_sqrt_n;
            }
            J[(size_t)a * N + b] = v;
            J[(size_t)b * N + a] = v;
        }
    }
    return 0;
}

/* --------------------------------------------------------------------------- exp */

/* exp(x) for x <= 0.  x = k ln2 + r with |r| <= ln2/2 (Cody-Waite: ln 2 split into
 * a 32-significant-bit head, so k * head is exact, and a tail); exp(r) by the
 * Taylor series to degree 13 in Horner form; result scaled by 2^k.  Values below
 * -708 return 0 (a weight below 2^-1021 cannot change any selection, see select). */
double mc3o_exp(double x)
{
    const double LOG2E = 0x1.71547652b82fep+0;
    const double LN2_HEAD = 0x1.62e42ff000000p-1;
    const double LN2_TAIL = -0x1.718432a1b0e26p-35;
    /* 1/n! rounded to nearest, n = 13 .. 2 */
    const double C13 = 0x1.6124613a86d09p-33, C12 = 0x1.1eed8eff8d898p-29;
    const double C11 = 0x1.ae64567f544e4p-26, C10 = 0x1.27e4fb7789f5cp-22;
    const double C9 = 0x1.71de3a556c734p-19, C8 = 0x1.a01a01a01a01ap-16;
    const double C7 = 0x1.a01a01a01a01ap-13, C6 = 0x1.6c16c16c16c17p-10;
    const double C5 = 0x1.1111111111111p-7, C4 = 0x1.5555555555555p-5;
    const double C3 = 0x1.5555555555555p-3, C2 = 0x1.0p-1;
    if (x != x) return x;
    if (x < -708.0) return 0.0;
    if (x > 709.0) return INFINITY;
    double kd = floor(x * LOG2E + 0.5);
    int k = (int)kd;
    double r = (x - kd * LN2_HEAD) - kd * LN2_TAIL;
    double p = C13;
    p = p * r + C12;
    p = p * r + C11;
    p = p * r + C10;
    p = p * r + C9;
    p = p * r + C8;
    p = p * r + C7;
    p = p * r + C6;
    p = p * r + C5;
    p = p * r + C4;
    p = p * r + C3;
    p = p * r + C2;
    p = p * r + 1.0;
    p = p * r + 1.0;
    uint64_t bits = (uint64_t)(k + 1023) << 52;   /* 2^k, a normal number here */
    double two_k;
    memcpy(&two_k, &bits, sizeof two_k);
    return p * two_k;
}

/* ------------------------------------------------------------------------- Floyd */

/* Floyd's k-of-N distinct-site draw, driven by the given words (k words):
 * for j = N-k .. N-1: t = randint(word, j+1); insert t unless already present,
 * else insert j.  member[0..N-1] receives 0/1. */
void mc3o_floyd_words(int N, int k, const uint32_t* words, uint8_t* member)
{
    memset(member, 0, (size_t)N);
    for (int idx = 0; idx < k; ++idx) {
        int j = N - k + idx;
        uint32_t t = mc3o_randint(words[idx], (uint32_t)(j + 1));
        if (member[t]) member[j] = 1;
        else member[t] = 1;
    }
}

/* ------------------------------------------------------------------------ energy */

/* E(s) = -scale * sum_{i<j} J_ij s_i s_j with J row-major N x N (only the strict
 * upper triangle is read), plain i-major double loop. */
double mc3o_energy(int N, const double* J, double scale, const int8_t* s)
{
    double sum = 0.0;
    for (int i = 0; i < N; ++i) {
        for (int j = i + 1; j < N; ++j) {
            double term = J[(size_t)i * N + j];
            if (s[i] != s[j]) term = -term;
            sum += term;
        }
    }
    return -(scale * sum);
}

/* Initial spins: bit i%32 of word i/32 of the INIT stream (step 0, edge 0);
 * a set bit means spin -1. */
void mc3o_init_spins(uint64_t seed, int N, uint32_t chain, int8_t* s)
{
    for (int i = 0; i < N; ++i) {
        uint32_t w = mc3o_word(seed, TAG_INIT, chain, 0u, 0u, (uint32_t)(i / 32));
        s[i] = ((w >> (i % 32)) & 1u) ? (int8_t)-1 : (int8_t)1;
    }
}

/* ------------------------------------------------------------------------ propose */

/* Flip set of edge e (1..M) of chain `chain` at `step`:
 * k_e = kmin + randint(word 0, kmax-kmin+1), then Floyd on words 1..k_e. */
int mc3o_edge_flips(uint64_t seed, uint32_t chain, uint32_t step, uint32_t edge,
                    int N, int kmin, int kmax, uint8_t* member)
{
    uint32_t w0 = mc3o_word(seed, TAG_EDGE, chain, step, edge, 0u);
    int k = kmin + (int)mc3o_randint(w0, (uint32_t)(kmax - kmin + 1));
    uint32_t* words = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(k > 0 ? k : 1));
    for (int idx = 0; idx < k; ++idx)
        words[idx] = mc3o_word(seed, TAG_EDGE, chain, step, edge, (uint32_t)(1 + idx));
    mc3o_floyd_words(N, k, words, member);
    free(words);
    return k;
}

/* Root position r in {0..M}: randint(ROOT word 0, M+1). */
int mc3o_root(uint64_t seed, uint32_t chain, uint32_t step, int M)
{
    return (int)mc3o_randint(mc3o_word(seed, TAG_ROOT, chain, step, 0u, 0u), (uint32_t)(M + 1));
}

/* Root position of the line-graph addition process: the number of the M additions
 * that went to the left end, addition j going left iff bit j%32 of ROOT word j/32
 * is set (j = 0..M-1). */
int mc3o_root_line(uint64_t seed, uint32_t chain, uint32_t step, int M)
{
    int k = 0;
    for (int j = 0; j < M; ++j) {
        uint32_t w = mc3o_word(seed, TAG_ROOT, chain, step, 0u, (uint32_t)(j / 32));
        k += (int)((w >> (j % 32)) & 1u);
    }
    return k;
}

/* A root law given by weights g_v >= 0 (v = 0..M), in fixed point: S = sum of g in
 * node order, q_v = floor(g_v / S * 2^52), and Q_v = q_0 + ... + q_v (written to
 * Qcum), so node v is the root with probability q_v / Q_M.  Returns -1 when a weight
 * is negative or not finite, or when every q_v is 0. */
int mc3o_root_table_prepare(int M, const double* g, uint64_t* Qcum)
{
    double S = 0.0;
    for (int v = 0; v <= M; ++v) {
        if (!(g[v] >= 0.0) || g[v] == INFINITY) return -1;
        S += g[v];
    }
    if (!(S > 0.0) || S == INFINITY) return -1;
    uint64_t acc = 0;
    for (int v = 0; v <= M; ++v) {
        acc += (uint64_t)floor(g[v] / S * 0x1.0p52);
        Qcum[v] = acc;
    }
    return acc > 0 ? 0 : -1;
}

/* Root position under a table law: u53 from ROOT words 0 and 1, threshold
 * t = floor(u53 W / 2^53) with W = Q_M, root = min { v : Q_v > t }. */
int mc3o_root_table(uint64_t seed, uint32_t chain, uint32_t step, int M, const uint64_t* Qcum)
{
    uint32_t w0 = mc3o_word(seed, TAG_ROOT, chain, step, 0u, 0u);
    uint32_t w1 = mc3o_word(seed, TAG_ROOT, chain, step, 0u, 1u);
    uint64_t u53 = mc3o_u53(w0, w1);
    unsigned __int128 prod = (unsigned __int128)u53 * (unsigned __int128)Qcum[M];
    uint64_t t = (uint64_t)(prod >> 53);
    int r = 0;
    while (Qcum[r] <= t) ++r;
    return r;
}

/* The table law's log-prior: log of the fixed-point root probability's numerator,
 * log((double) q_v) (q_v = 0 gives -infinity: the node is never chosen). */
void mc3o_log_prior_table(int M, const uint64_t* Qcum, double* out)
{
    for (int v = 0; v <= M; ++v) {
        uint64_t q = Qcum[v] - (v ? Qcum[v - 1] : 0u);
        out[v] = q ? log((double)q) : -INFINITY;
    }
}

/* log C(M, v) for v = 0..M: the line process's log-prior, lgamma(M+1) - lgamma(v+1)
 * - lgamma(M-v+1) evaluated left to right. */
void mc3o_log_prior_line(int M, double* out)
{
    for (int v = 0; v <= M; ++v)
        out[v] = lgamma((double)M + 1.0) - lgamma((double)v + 1.0) - lgamma((double)(M - v) + 1.0);
}

/* Node configurations of the tree (M+1 nodes, arity a; a = M is the star) generated
 * from the current state s sitting at node r: node v is s with the flip sets of the
 * edges on the path between r and v flipped.  With path(v) = the edges from node 0
 * down to v, that set is path(r) xor path(v) (the common part cancels).  For the
 * star: r = 0 gives hub = s, leaf e = s^F_e; r >= 1 gives leaf r = s, hub = s^F_r,
 * leaf e = s^F_r^F_e.  flips: [(M+1) x N], row 0 unused; nodes: [(M+1) x N] int8. */
void mc3o_build_nodes(int N, int M, int arity, int r, const int8_t* s, const uint8_t* flips, int8_t* nodes)
{
    uint8_t* path = (uint8_t*)calloc((size_t)(M + 1) * N, 1);
    for (int v = 1; v <= M; ++v) {
        int par = (v - 1) / arity;
        for (int i = 0; i < N; ++i)
            path[(size_t)v * N + i] = path[(size_t)par * N + i] ^ flips[(size_t)v * N + i];
    }
    for (int v = 0; v <= M; ++v) {
        for (int i = 0; i < N; ++i) {
            int flip = path[(size_t)r * N + i] ^ path[(size_t)v * N + i];
            nodes[(size_t)v * N + i] = flip ? (int8_t)(-s[i]) : s[i];
        }
    }
    free(path);
}

/* ------------------------------------------------------------------------ select */

typedef struct {
    int32_t r;          /* root position (position of the state the graph was generated from) */
    int32_t vstar;      /* selected node */
    double e_cur;       /* energy of the selected node (the new current state) */
    double e_bar;       /* node-weighted energy sum_v P_node(v) E_v */
    double margin;      /* distance of the draw to the selected interval's edges, in units of W */
    uint64_t wsum;      /* W: sum of the fixed-point weights */
} mc3o_rec;

/* MCMCMC node rule for a self-thermalising graph:
 * P_node(v) proportional to exp(-beta (E_v - Emin)).
 * Weights w_v = exp(-(beta*(E_v - Emin))) in FP64, then q_v = floor(w_v * 2^52)
 * (exact integers), Q_v = inclusive prefix sum, W = Q_M, threshold
 * t = floor(u53 * W / 2^53), selected v* = min { v : Q_v > t }.
 * log_prior (may be NULL) adds log g_v to the exponent for non-uniform P_gen. */
int mc3o_select_mcmcmc(int nodes, const double* E, const double* log_prior, double beta,
                       uint64_t u53, double* e_bar, double* margin, uint64_t* wsum)
{
    double emin = E[0];
    for (int v = 1; v < nodes; ++v) if (E[v] < emin) emin = E[v];
    double* w = (double*)malloc(sizeof(double) * (size_t)nodes);
    double lmax = -INFINITY;
    for (int v = 0; v < nodes; ++v) {
        double l = -(beta * (E[v] - emin));
        if (log_prior) l = l + log_prior[v];
        w[v] = l;
        if (l > lmax) lmax = l;
    }
    for (int v = 0; v < nodes; ++v) w[v] = mc3o_exp(w[v] - lmax);
    uint64_t Wq = 0;
    uint64_t* Q = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)nodes);
    for (int v = 0; v < nodes; ++v) {
        uint64_t q = (uint64_t)floor(w[v] * 0x1.0p52);
        Wq += q;
        Q[v] = Wq;
    }
    unsigned __int128 prod = (unsigned __int128)u53 * (unsigned __int128)Wq;
    uint64_t t = (uint64_t)(prod >> 53);
    int vs = 0;
    while (Q[vs] <= t) ++vs;
    uint64_t lo = vs ? Q[vs - 1] : 0u;
    uint64_t d1 = t - lo, d2 = Q[vs] - t;
    *margin = (double)(d1 < d2 ? d1 : d2) / (double)Wq;
    double num = 0.0, den = 0.0;
    for (int v = 0; v < nodes; ++v) { num += w[v] * E[v]; den += w[v]; }
    *e_bar = num / den;
    *wsum = Wq;
    free(w);
    free(Q);
    return vs;
}

/* Metropolis rate min(1, exp(-beta dE)) for one proposal.  Accept iff dE <= 0 or
 * u < exp(-(beta*dE)), u = u53 / 2^53. */
int mc3o_accept_metropolis(double e_cur, double e_new, double beta, uint64_t u53, double* margin)
{
    double dE = e_new - e_cur;
    if (dE <= 0.0) { *margin = INFINITY; return 1; }
    double w = mc3o_exp(-(beta * dE));
    double u = (double)u53 * 0x1.0p-53;
    *margin = fabs(u - w);
    return u < w;
}

/* ------------------------------------------------- state-dependent proposals */

/* Site weights of the biased single-site proposal from state s (Sec. "Problem
 * statement": the two-body proposal may be any ergodic law; here it depends on the
 * state).  Site i is proposed with probability proportional to exp(-alpha dE_i), dE_i
 * = E(s with i flipped) - E(s) = 2 scale s_i h_i, h_i = sum_j J_ij s_j (plain sum).  In
 * fixed point: a_i = -(alpha ((2 scale) (s_i h_i))), amax = max a, q_i =
 * floor(exp(a_i - amax) 2^52) (every q_i of the largest a_i is 2^52), written to q;
 * returns W = sum q_i in site order. */
uint64_t mc3o_site_weights(int N, const double* J, double scale, double alpha, const int8_t* s, uint64_t* q)
{
    double* a = (double*)malloc(sizeof(double) * (size_t)N);
    double amax = -INFINITY;
    for (int i = 0; i < N; ++i) {
        double h = 0.0;
        for (int j = 0; j < N; ++j) h += J[(size_t)i * N + j] * (double)s[j];
        double x = (double)s[i] * h;
        a[i] = -(alpha * ((2.0 * scale) * x));
        if (a[i] > amax) amax = a[i];
    }
    uint64_t W = 0;
    for (int i = 0; i < N; ++i) {
        q[i] = (uint64_t)floor(mc3o_exp(a[i] - amax) * 0x1.0p52);
        W += q[i];
    }
    free(a);
    return W;
}

/* The site drawn from weights q (total W) by the 53-bit uniform u53:
 * t = floor(u53 W / 2^53), site = min { i : q_0 + .. + q_i > t }. */
int mc3o_draw_site(int N, const uint64_t* q, uint64_t W, uint64_t u53)
{
    unsigned __int128 prod = (unsigned __int128)u53 * (unsigned __int128)W;
    uint64_t t = (uint64_t)(prod >> 53);
    uint64_t Q = 0;
    for (int i = 0; i < N; ++i) {
        Q += q[i];
        if (Q > t) return i;
    }
    return N - 1;
}

/* Node rule with generation-probability ratios (App. "Markov chain of graphs of
 * configurations", Eq. eq_det_balance_graph_solution): P_node(v) proportional to
 * exp(-beta E_v) rho_v, rho_v = P_gen(T|c_v) / P_gen(T|c_0).  Fixed point:
 * y_v = exp(-(beta (E_v - Emin))) rho_v, w_v = y_v / max y, q_v = floor(w_v 2^52),
 * Q_v inclusive sums in node order, t = floor(u53 W / 2^53), v* = min{v : Q_v > t};
 * margin and node-weighted energy as mc3o_select_mcmcmc. */
int mc3o_select_ratio(int nodes, const double* E, const double* rho, double beta, uint64_t u53,
                      double* e_bar, double* margin, uint64_t* wsum)
{
    double emin = E[0];
    for (int v = 1; v < nodes; ++v) if (E[v] < emin) emin = E[v];
    double* w = (double*)malloc(sizeof(double) * (size_t)nodes);
    double ymax = 0.0;
    for (int v = 0; v < nodes; ++v) {
        w[v] = mc3o_exp(-(beta * (E[v] - emin))) * rho[v];
        if (w[v] > ymax) ymax = w[v];
    }
    for (int v = 0; v < nodes; ++v) w[v] = w[v] / ymax;
    uint64_t Wq = 0;
    uint64_t* Q = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)nodes);
    for (int v = 0; v < nodes; ++v) {
        Wq += (uint64_t)floor(w[v] * 0x1.0p52);
        Q[v] = Wq;
    }
    unsigned __int128 prod = (unsigned __int128)u53 * (unsigned __int128)Wq;
    uint64_t t = (uint64_t)(prod >> 53);
    int vs = 0;
    while (Q[vs] <= t) ++vs;
    uint64_t lo = vs ? Q[vs - 1] : 0u;
    uint64_t d1 = t - lo, d2 = Q[vs] - t;
    *margin = (double)(d1 < d2 ? d1 : d2) / (double)Wq;
    double num = 0.0, den = 0.0;
    for (int v = 0; v < nodes; ++v) { num += w[v] * E[v]; den += w[v]; }
    *e_bar = num / den;
    *wsum = Wq;
    free(w);
    free(Q);
    return vs;
}

/* One step of one chain with the biased single-site proposal on the star (uniform root
 * r ~ U{0..M}, App. "General graph populating process"): r = 0: the hub is the current
 * state s; r >= 1: s is leaf r and the hub is s with site i_r flipped, i_r drawn from
 * the weights of s; every other leaf e is the hub with site i_e flipped, i_e drawn from
 * the weights of the hub.  The site of edge e is drawn with u53 of words 0, 1 of the
 * edge stream (tag 3, edge e).  With a uniform root, P_gen(T|c_v) relative to the hub
 * is rho_v = p_{i_v}(c_v) / p_{i_v}(hub) for leaf v (c_v generates the hub through
 * site i_v; every other edge is generated from the hub either way), taken in fixed
 * point as ((q_{i_v}(c_v) W(hub)) / (q_{i_v}(hub) W(c_v))), rho_hub = 1.  When the hub
 * cannot generate leaf r (q_{i_r}(hub) = 0) only node r has a nonzero generation
 * probability: the chain stays (v* = r, margin infinite, e_bar = E_r).
 * nodes: [(M+1) x N] out; E: [M+1] out (plain pair sums); rho [M+1] out. */
int mc3o_biased_step(int N, int M, const double* J, double scale, double alpha, double beta, uint64_t seed,
                     uint32_t chain, uint32_t step, const int8_t* s, int8_t* nodes, double* E, double* rho,
                     int* r_out, double* e_bar, double* margin)
{
    uint64_t* qs = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)N);
    uint64_t* qh = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)N);
    uint64_t* qv = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)N);
    int* site = (int*)malloc(sizeof(int) * (size_t)(M + 1));
    const int r = mc3o_root(seed, chain, step, M);
    int8_t* hub = nodes;
    memcpy(hub, s, (size_t)N);
    if (r >= 1) {
        uint64_t Ws = mc3o_site_weights(N, J, scale, alpha, s, qs);
        uint64_t u = mc3o_u53(mc3o_word(seed, TAG_EDGE, chain, step, (uint32_t)r, 0u),
                              mc3o_word(seed, TAG_EDGE, chain, step, (uint32_t)r, 1u));
        site[r] = mc3o_draw_site(N, qs, Ws, u);
        hub[site[r]] = (int8_t)-hub[site[r]];
    }
    uint64_t Wh = mc3o_site_weights(N, J, scale, alpha, hub, qh);
    for (int e = 1; e <= M; ++e) {
        if (e != r) {
            uint64_t u = mc3o_u53(mc3o_word(seed, TAG_EDGE, chain, step, (uint32_t)e, 0u),
                                  mc3o_word(seed, TAG_EDGE, chain, step, (uint32_t)e, 1u));
            site[e] = mc3o_draw_site(N, qh, Wh, u);
        }
        int8_t* leaf = nodes + (size_t)e * N;
        memcpy(leaf, hub, (size_t)N);
        leaf[site[e]] = (int8_t)-leaf[site[e]];
    }
    for (int v = 0; v <= M; ++v) E[v] = mc3o_energy(N, J, scale, nodes + (size_t)v * N);
    rho[0] = 1.0;
    for (int v = 1; v <= M; ++v) {
        uint64_t Wv = mc3o_site_weights(N, J, scale, alpha, nodes + (size_t)v * N, qv);
        double num = (double)qv[site[v]] * (double)Wh;
        double den = (double)qh[site[v]] * (double)Wv;
        rho[v] = num / den;   /* den = 0 only at v = r: handled below */
    }
    uint32_t w0 = mc3o_word(seed, TAG_SELECT, chain, step, 0u, 0u);
    uint32_t w1 = mc3o_word(seed, TAG_SELECT, chain, step, 0u, 1u);
    int vs;
    uint64_t wsum;
    if (r >= 1 && qh[site[r]] == 0) {
        vs = r;
        *margin = INFINITY;
        *e_bar = E[r];
    } else {
        vs = mc3o_select_ratio(M + 1, E, rho, beta, mc3o_u53(w0, w1), e_bar, margin, &wsum);
    }
    *r_out = r;
    free(qs); free(qh); free(qv); free(site);
    return vs;
}

/* ------------------------------------------------------------------------ run */

typedef struct {
    int32_t N, M, chains, kmin, kmax;
    int32_t rule;          /* 0 = MCMCMC, 1 = METROPOLIS (M must be 1) */
    uint32_t chain_base;   /* global index of chain 0 (RNG counter) */
    uint32_t pad;
    uint64_t seed;
    double scale;          /* energy scale: E = -scale * sum_{i<j} J_ij s_i s_j */
    int32_t arity;         /* tree arity (parent of v is (v-1)/arity); 0 = M (the star) */
    int32_t law;           /* 0 = uniform root, 1 = line-graph addition process (arity 1), 2 = table,
                              3 = star with the state-dependent single-site proposal (mc3o_biased_step) */
    int32_t pad2;
    const double* table;   /* law 2: root weights g_0..g_M */
    double alpha;          /* law 3: bias of the state-dependent single-site proposal */
} mc3o_cfg;

/* Run nsteps steps starting at global step step0 for every chain.
 *   spins  [chains][N] in/out, e_cur [chains] in/out (energy of the current state).
 *   beta   [nsteps] inverse temperature per step.
 *   rec    [nsteps][chains] records (may be NULL).
 *   node_e [nsteps][chains][M+1] energies of every node (may be NULL).
 *   forced [nsteps][chains] node to take instead of the drawn one, -1 = none
 *          (guided replay at steps where the compared path reported a near-tie;
 *          may be NULL).
 * Every node energy is recomputed from its configuration by the plain pair sum,
 * including the current state's.  Returns 0, or -1 on a bad configuration. */
int mc3o_run(const mc3o_cfg* cfg, const double* J, int8_t* spins, double* e_cur,
             uint64_t step0, int64_t nsteps, const double* beta,
             mc3o_rec* rec, double* node_e, const int32_t* forced)
{
    const int N = cfg->N, M = cfg->M;
    if (N < 2 || M < 1 || cfg->chains < 1 || cfg->kmin < 1 || cfg->kmax < cfg->kmin || cfg->kmax > N) return -1;
    if (cfg->rule == 1 && M != 1) return -1;
    const int arity = cfg->arity > 0 ? cfg->arity : M;
    if (arity > M || cfg->law < 0 || cfg->law > 3 || (cfg->law == 1 && arity != 1)) return -1;
    if (cfg->law == 3 && (arity != M || cfg->kmin != 1 || cfg->kmax != 1 || cfg->rule != 0)) return -1;
    if (cfg->law == 2 && !cfg->table) return -1;
    double* log_prior = NULL;
    uint64_t* Qcum = NULL;
    if (cfg->law == 1) {
        log_prior = (double*)malloc(sizeof(double) * (size_t)(M + 1));
        mc3o_log_prior_line(M, log_prior);
    } else if (cfg->law == 2) {
        log_prior = (double*)malloc(sizeof(double) * (size_t)(M + 1));
        Qcum = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(M + 1));
        if (mc3o_root_table_prepare(M, cfg->table, Qcum) != 0) {
            free(log_prior);
            free(Qcum);
            return -1;
        }
        mc3o_log_prior_table(M, Qcum, log_prior);
    }
    uint8_t* flips = (uint8_t*)malloc((size_t)(M + 1) * N);
    int8_t* nodes = (int8_t*)malloc((size_t)(M + 1) * N);
    double* E = (double*)malloc(sizeof(double) * (size_t)(M + 1));
    double* rho_buf = (double*)malloc(sizeof(double) * (size_t)(M + 1));   /* law 3: rho per node */
    for (int64_t ts = 0; ts < nsteps; ++ts) {
        uint32_t step = (uint32_t)(step0 + (uint64_t)ts);
        for (int c = 0; c < cfg->chains; ++c) {
            uint32_t gc = cfg->chain_base + (uint32_t)c;
            int8_t* s = spins + (size_t)c * N;
            if (cfg->law == 3) {
                int r3, vs3;
                double eb3, mg3;
                vs3 = mc3o_biased_step(N, M, J, cfg->scale, cfg->alpha, beta[ts], cfg->seed, gc, step, s, nodes, E,
                                       rho_buf, &r3, &eb3, &mg3);
                if (forced && forced[(size_t)ts * cfg->chains + c] >= 0) vs3 = forced[(size_t)ts * cfg->chains + c];
                if (node_e) memcpy(node_e + ((size_t)ts * cfg->chains + c) * (M + 1), E, sizeof(double) * (size_t)(M + 1));
                memcpy(s, nodes + (size_t)vs3 * N, (size_t)N);
                e_cur[c] = E[vs3];
                if (rec) {
                    mc3o_rec* o = rec + (size_t)ts * cfg->chains + c;
                    o->r = r3; o->vstar = vs3; o->e_cur = E[vs3]; o->e_bar = eb3; o->margin = mg3; o->wsum = 0;
                }
                continue;
            }
            int r = 0;
            if (cfg->rule != 1) {
                if (cfg->law == 1)
                    r = mc3o_root_line(cfg->seed, gc, step, M);
                else if (cfg->law == 2)
                    r = mc3o_root_table(cfg->seed, gc, step, M, Qcum);
                else
                    r = mc3o_root(cfg->seed, gc, step, M);
            }
            memset(flips, 0, (size_t)N);
            for (int e = 1; e <= M; ++e)
                mc3o_edge_flips(cfg->seed, gc, step, (uint32_t)e, N, cfg->kmin, cfg->kmax, flips + (size_t)e * N);
            mc3o_build_nodes(N, M, arity, r, s, flips, nodes);
            for (int v = 0; v <= M; ++v) E[v] = mc3o_energy(N, J, cfg->scale, nodes + (size_t)v * N);
            uint32_t w0 = mc3o_word(cfg->seed, TAG_SELECT, gc, step, 0u, 0u);
            uint32_t w1 = mc3o_word(cfg->seed, TAG_SELECT, gc, step, 0u, 1u);
            uint64_t u53 = mc3o_u53(w0, w1);
            int vs;
            double ebar, margin;
            uint64_t wsum = 0;
            if (cfg->rule == 1) {
                int acc = mc3o_accept_metropolis(E[0], E[1], beta[ts], u53, &margin);
                vs = acc ? 1 : 0;
                ebar = E[vs];
            } else {
                vs = mc3o_select_mcmcmc(M + 1, E, log_prior, beta[ts], u53, &ebar, &margin, &wsum);
            }
            if (forced && forced[(size_t)ts * cfg->chains + c] >= 0)
                vs = forced[(size_t)ts * cfg->chains + c];
            if (node_e) memcpy(node_e + ((size_t)ts * cfg->chains + c) * (M + 1), E, sizeof(double) * (size_t)(M + 1));
            memcpy(s, nodes + (size_t)vs * N, (size_t)N);
            e_cur[c] = E[vs];
            if (rec) {
                mc3o_rec* o = rec + (size_t)ts * cfg->chains + c;
                o->r = r; o->vstar = vs; o->e_cur = E[vs]; o->e_bar = ebar;
                o->margin = margin; o->wsum = wsum;
            }
        }
    }
    free(flips); free(nodes); free(E); free(rho_buf); free(log_prior); free(Qcum);
    return 0;
}

/* ------------------------------------------------------------------------ sets */

/* The set variant's generation probability, from its definition (Sec. "Stochastic
 * generation of the set"): a set grows from a nonempty subset X of S = {0..n-1} by
 * additions; each addition chooses a parent uniformly among the current elements and
 * generates the new element e with probability G[e*n + parent] (G[e][parent] =
 * P_gen(e | parent)); S is reached when the n - |X| additions bring exactly the
 * elements of S \ X, in some order.  P_gen(S | X) is the sum over the orders
 * (e_1, .., e_r) of S \ X of prod_j (1/|X_j|) sum_{p in X_j} G[e_j][p], with
 * X_j = X + {e_1 .. e_(j-1)}; every order is enumerated explicitly (r <= 10).
 * Returns -1 for an empty X, r > 10, or n > 30. */
double mc3o_set_gen_brute(int n, const double* G, uint32_t X, int* status)
{
    *status = 0;
    if (n < 1 || n > 30 || X == 0u) { *status = -1; return 0.0; }
    int add[32], r = 0;
    for (int e = 0; e < n; ++e) if (!((X >> e) & 1u)) add[r++] = e;
    if (r == 0) return 1.0;
    if (r > 10) { *status = -1; return 0.0; }
    /* orders in lexicographic order of index permutations */
    int perm[32];
    for (int i = 0; i < r; ++i) perm[i] = i;
    double total = 0.0;
    for (;;) {
        uint32_t cur = X;
        int size = 0;
        for (int e = 0; e < n; ++e) size += (int)((X >> e) & 1u);
        double prob = 1.0;
        for (int j = 0; j < r; ++j) {
            int e = add[perm[j]];
            double s = 0.0;
            for (int p = 0; p < n; ++p)
                if ((cur >> p) & 1u) s += G[(size_t)e * n + p];
            prob *= s / (double)size;
            cur |= 1u << e;
            ++size;
        }
        total += prob;
        /* next permutation */
        int i = r - 2;
        while (i >= 0 && perm[i] > perm[i + 1]) --i;
        if (i < 0) break;
        int k = r - 1;
        while (perm[k] < perm[i]) --k;
        int t = perm[i]; perm[i] = perm[k]; perm[k] = t;
        for (int a = i + 1, b = r - 1; a < b; ++a, --b) { t = perm[a]; perm[a] = perm[b]; perm[b] = t; }
    }
    return total;
}
