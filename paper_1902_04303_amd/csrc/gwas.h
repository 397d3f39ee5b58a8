// Encrypted modified semi-parallel GWAS circuit (device) and client-side packing.
#pragma once

#include <map>
#include <tuple>

#include "evaluator.h"

namespace gck {

// degree-7 sigmoid magnitudes in powers of x/8 (paper: Methods, eq. sigma7)
constexpr double kSigma7C1 = 1.73496;
constexpr double kSigma7C3 = 4.19407;
constexpr double kSigma7C5 = 5.43402;
constexpr double kSigma7C7 = 2.50739;

struct Layout {
    int N = 0, n = 0, k = 0, m = 0, R = 0, blocks = 0, tau = 0, n_batches = 0;
};

inline int a_index(int k, int j, int l) {   // (j <= l) in row-major upper-triangle order
    int idx = 0;
    for (int a = 0; a < j; ++a) idx += k - a;
    return idx + (l - j);
}

struct EncInput {
    Layout lay;
    int kappa = 0;
    std::vector<Ct> x;   // k ciphertexts, depth 0
    Ct y;                // depth 0
    std::vector<Ct> A;   // k(k+1)/2, depth 0, scale R Delta_0
    Ct S;                // batched: n_batches ciphertexts at snp_depth(kappa) (data empty when spilled)
    u64 *S_host = nullptr;   // the SNP batches in pinned host memory after a spill
    // M-materialised layout (set by attach_m): X^T in REP form, X_ij replicated, stored column-major
    // ([j][i], n k ciphertexts at snp_depth + 1), and the REP rows of every SNP batch ([b][i], n_batches n
    // ciphertexts at snp_depth + 2).  When present the circuit computes S' = M S by CP-REP-MatMult.
    Ct Xrep, S_rep;
    ~EncInput() {
        if (S_host) (void)hipHostFree(S_host);
    }
};
// copy SNP batches [b0, b0 + cnt) of `in` (device or spilled host copy) into slots di.. of dst, on stream st
void fetch_snp(ckks_ctx &c, const EncInput &in, int b0, int cnt, ckks_ct &dst, int di, hipStream_t st);
// move the SNP batches to pinned host memory (they are streamed back chunk by chunk when used)
void spill_snp(ckks_ctx &c, EncInput &in);

struct EncOutput {
    std::vector<Ct> beta;
    Ct w, w_inv, z_proj, u;   // w and w_inv empty for kappa = 1 (public constants)
    std::vector<Ct> S_proj, num, den_even, den_odd;   // one batched ciphertext per chunk
    // after run_divide, per chunk of cnt SNP batches: 2 cnt ciphertexts, the even SNPs' then the odd SNPs'
    // (b': real part of the even half, imaginary part of the odd half; err': real part)
    std::vector<Ct> div_b, div_inv;
    Ct m_cols;   // M-materialised layout: Dup(M_i), i < n (at the SNP depth + 2)
    int chunk = 0;
};

// what the per-batch part needs from the fixed part (batch of one per job, or one per SNP batch)
struct FixedOut {
    std::vector<Ct> r_s;   // r_j = (X A)_{:, j} at the SNP depth
    std::vector<Ct> x_c;   // x_j at the SNP depth + 2
    int K = 0;             // width of the packed projection (0: one colSum and broadcast per covariate)
    std::vector<Ct> z_d;   // packed projection: Rot(Z_t, -t) at the SNP depth, t < K
    std::vector<Ct> x_d;   // packed projection: X_t at the SNP depth + 2, t < K
    Ct u_s, w_s;           // u = w z' at the SNP depth + 3, w at + 4 (w_s empty when w is public: kappa = 1)
    std::vector<Ct> hold;  // batches that r_s and x_c may be views of
    Ct m_cols;             // M-materialised layout: Dup(M_i), i < n, at the SNP depth + 2
};
struct BatchOut {
    Ct sp, num, de, dodd;
};

int circuit_levels(int kappa);
int snp_depth(int kappa);
Layout make_layout(int n_ring, int n, int k, int m);
// Rotations of the rotate-and-sum over R = 2^r slots, by shared key switch: {s, 2s, .., (m - 1) s} with
// m = min(radix, R / s) for s = 1, then s times the previous m.  Radix 4 gives {s, 2s, 3s} for
// s = 1, 4, 16, .. and a last {s} when r is odd.  The fixed part (few ciphertexts per call at high
// levels, so key reads weigh more) uses radix 8, 3 key switches for R = 256 (measured: radix 4, 8 and 16
// took 65.4, 64.4 and 64.8 ms per paper-size job); the per-SNP-batch part (many ciphertexts per call,
// ModUp and ModDown weigh most) uses radix 16, 2 key switches for R = 256.
constexpr int kFixedRadix = 8, kBatchRadix = 16;
std::vector<std::vector<i64>> rotation_groups(int R, int radix);
// Packed projection of the SNP batches (all k covariates' column sums in one ciphertext): its width K, the
// smallest power of two >= k, or 0 where it does not apply (k < 2, K above min(kBatchRadix, R), or
// n + K - 1 > R: the rows that its products and stride sums wrap onto must be padding rows)
int diag_width(const Layout &lay);
// The rotations of sum_{u < R/K} Rot(a, K u) by shared key switch: the multiples of K in the first group of
// rotation_groups(R, radix), then its other groups (every rotation is one of rotation_groups(R, radix))
std::vector<std::vector<i64>> stride_groups(int R, int K, int radix);
// Galois elements of the rotations of rotation_groups(R, 8) and rotation_groups(R, 16) in both
// directions (each once, in that order), then conjugation
std::vector<u64> required_galois(int n, int R);
// K: the packed projection's width (diag_width), 0 for one colSum and broadcast per covariate
void run_fixed(ckks_ctx &c, int R, int k, int kappa, const std::vector<const ckks_ct *> &x, const ckks_ct &y,
               const std::vector<const ckks_ct *> &A, int ds, FixedOut &fx, EncOutput &rep, int K);
BatchOut run_batch(ckks_ctx &c, int R, int k, const FixedOut &fx, const ckks_ct &S);
void run_circuit(ckks_ctx &c, const EncInput &in, EncOutput &out, int chunk);
void run_multi(ckks_ctx &c, const std::vector<const EncInput *> &jobs, std::vector<EncOutput> &outs, int chunk);
// SNP batches per pass of a large job in the batched form (its transient key-switch buffers, about 20 MB per
// batch at the per-batch part's levels, stay near 5 GB)
constexpr int kMultiChunk = 256;
constexpr size_t kMaxFixedJobs = 8;   // jobs whose fixed parts run as one batch in run_multi
// building blocks shared with the server
struct WorkItem {
    const EncInput *in;
    const FixedOut *fx;
    EncOutput *out;
    int batch;
};
// jobs that share launches: same R, k, kappa and packed-projection width
std::tuple<int, int, int, int> bucket_of(const EncInput &in);
void fixed_for_jobs(ckks_ctx &c, const std::vector<const EncInput *> &jobs, std::vector<FixedOut> &fxs,
                    std::vector<EncOutput> &reps);
void chunk_for_jobs(ckks_ctx &c, const std::vector<WorkItem> &items);
std::unique_ptr<EncInput> pack_encrypt(ckks_ctx &c, const double *X, const double *y, const uint8_t *S, int n, int k,
                                       int m, int kappa, u64 enc_seed);

size_t input_footprint(const ckks_ctx &c, const EncInput &in);

// homomorphic division (b' and err' as ciphertexts), kDivIters Newton steps from guess 1
constexpr int kDivIters = 5;
int div_levels();
void run_divide(ckks_ctx &c, EncOutput &out, const ckks_ct &v);
Ct pack_normalisers(ckks_ctx &c, const uint8_t *S, int n, int m, int kappa, u64 enc_seed);

// M-materialised layout: depths of the REP inputs, their client-side packing, and S' of a chunk
int m_xrep_depth(int kappa);
int m_srep_depth(int kappa);
void attach_m(ckks_ctx &c, EncInput &in, Ct xrep_row_major, Ct srep);
void pack_encrypt_m(ckks_ctx &c, EncInput &in, const double *X, const uint8_t *S, u64 enc_seed);
Ct batch_front_m(ckks_ctx &c, const FixedOut &fx, const ckks_ct &S_rep_chunk);

}  // namespace gck

struct gwas_enc_input {
    ckks_ctx *ctx;
    std::unique_ptr<gck::EncInput> in;
};

struct gwas_enc_output {
    ckks_ctx *ctx;
    gck::EncOutput out;
    gck::Layout lay;
};

// gwas_semiparallel of one input shape captured as a HIP graph: the captured call's input (a private
// copy, refilled by set_input), its output (rewritten by every replay) and every pool block the call
// used, reserved for the graph until it is destroyed.
struct gwas_graph {
    ckks_ctx *ctx = nullptr;
    std::unique_ptr<gck::EncInput> slot;
    std::unique_ptr<gwas_enc_output> out;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<std::pair<void *, size_t>> main_blocks, aux_blocks;
    int chunk = 0;
    ~gwas_graph();
};
namespace gck {
std::unique_ptr<gwas_graph> capture_circuit(ckks_ctx &c, const EncInput &in, int chunk);
// autotuner over schedules that leave every ciphertext bit-identical (chunk size, one or two streams)
struct TuneResult {
    ckks_ctx::Schedule best;
    double ms_default = 0;
    int candidates = 0;
};
TuneResult tune_circuit(ckks_ctx &c, const EncInput &in, int reps);
std::tuple<int, int, int, int> schedule_key(const EncInput &in);
void graph_set_input(gwas_graph &g, const EncInput &in);
void graph_launch(gwas_graph &g);
}  // namespace gck
