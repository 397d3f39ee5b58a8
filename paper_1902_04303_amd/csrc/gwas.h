// Encrypted modified semi-parallel GWAS circuit (device) and client-side packing.
#pragma once

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
    Ct S;                // batched: n_batches ciphertexts at depth 7 kappa
};

struct EncOutput {
    std::vector<Ct> beta;
    Ct w, w_inv, z_proj, u;
    std::vector<Ct> S_proj, num, den_even, den_odd;   // one batched ciphertext per chunk
    int chunk = 0;
};

int circuit_levels(int kappa);
int snp_depth(int kappa);
Layout make_layout(int n_ring, int n, int k, int m);
std::vector<u64> required_galois(const ckks_ctx &c, int R);
void run_circuit(ckks_ctx &c, const EncInput &in, EncOutput &out, int chunk);
std::unique_ptr<EncInput> pack_encrypt(ckks_ctx &c, const double *X, const double *y, const uint8_t *S, int n, int k,
                                       int m, int kappa, u64 enc_seed);

}  // namespace gck
