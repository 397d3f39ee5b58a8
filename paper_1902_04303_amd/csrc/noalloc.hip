// The relinearised product without device allocation (ckks_mul_noalloc): the same operation and kernels
// as ckks_mul, with every intermediate buffer (tensor, ModUp digits, key-switch accumulators, the limbs of
// the division by P q_{l-1}, the product before it is copied into the caller's ciphertext) carved from one
// file-scope device array.  Each GPU holds its own copy of the array from module load until the process
// ends; every call on a GPU shares it, so calls that overlap on one GPU (two host threads, or two
// contexts on different streams) race and must be serialised by the caller.  No buffer of the product is
// read before it is written, so nothing in the array has to start at zero and the last call's contents
// are harmless.
#include <map>
#include <mutex>

#include "evaluator.h"

namespace {

constexpr size_t kScratchBytes = (size_t)CKKS_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size must keep 256-byte blocks");

static __device__ __align__(256) uint64_t scratch[kScratchBytes / 8];

std::mutex g_mu;
std::map<int, void *> g_dev_ptr;   // device ordinal -> device address of that device's scratch

// Device address of the current device's scratch.  In host code `scratch` names a host-side stand-in,
// never device memory: only the address hipGetSymbolAddress returns (taken once per device, with that
// device current) is passed to kernels and copies.
void *scratch_ptr() {
    int dev = 0;
    GCK_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_dev_ptr.find(dev);
    if (it != g_dev_ptr.end()) return it->second;
    void *p = nullptr;
    GCK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw gck::Error(CKKS_E_HIP, "hipGetSymbolAddress returned no address for the scratch region");
    g_dev_ptr.emplace(dev, p);
    return p;
}

size_t blk(size_t words) { return (words * 8 + 255) & ~size_t(255); }

}  // namespace

namespace gck {

void noalloc_init() { (void)scratch_ptr(); }

size_t noalloc_max_bytes() { return kScratchBytes; }

// Bytes the product takes from the arena, in the order mul_sum and its fused relinearisation and rescale
// take their buffers (the arena gives back only its most recent block, so every one of them counts).
size_t mul_noalloc_bytes(const ckks_ctx &c, int count, int l) {
    const size_t N = (size_t)c.p.n;
    const int a = c.p.alpha, nt = l + a, rows = 2 * count;
    const size_t K = (size_t)c.ks_levels.at(l).K;
    return blk((size_t)count * 3 * l * N)        // tensor d0, d1, d2
           + blk((size_t)rows * (l - 1) * N)     // the product
           + blk((size_t)count * l * N)          // ModUp: coefficient limbs
           + blk((size_t)count * K * N)          // ModUp: digits at every target
           + blk((size_t)count * 2 * nt * N)     // inner-product accumulators
           + blk((size_t)rows * (a + 1) * N);    // the division by P q_{l-1}: its alpha + 1 limbs
}

void mul_noalloc(ckks_ctx &c, const ckks_ct &a, const ckks_ct &b, ckks_ct &out) {
    if (a.depth != b.depth) throw Error(CKKS_E_PARAM_MISMATCH, "product operands at different depths");
    if (a.limbs < 2) throw Error(CKKS_E_LEVEL, "no limb left to rescale");
    const int count = std::max(a.count, b.count);
    if (count % a.count || count % b.count) throw Error(CKKS_E_PARAM_MISMATCH, "batch counts differ");
    if (out.count != count || out.depth != a.depth + 1 || out.limbs != a.limbs - 1)
        throw Error(CKKS_E_PARAM_MISMATCH, "output must hold " + std::to_string(count) +
                                               " ciphertexts at depth " + std::to_string(a.depth + 1));
    const auto overlaps = [&](const ckks_ct &x) {
        return out.data.ptr < x.data.ptr + x.data.words && x.data.ptr < out.data.ptr + out.data.words;
    };
    if (overlaps(a) || overlaps(b)) throw Error(CKKS_E_INVALID_ARG, "output aliases an operand");
    const size_t need = mul_noalloc_bytes(c, count, a.limbs);
    if (need > kScratchBytes)
        throw Error(CKKS_E_INVALID_ARG, "product of " + std::to_string(count) + " ciphertexts at " +
                                            std::to_string(a.limbs) + " limbs needs " + std::to_string(need) +
                                            " bytes of scratch, above the maximum of " +
                                            std::to_string(kScratchBytes) + " bytes");
    std::unique_ptr<Pool> other = Pool::arena(scratch_ptr(), kScratchBytes);
    other->stream = c.stream;
    struct Swap {
        ckks_ctx &c;
        std::unique_ptr<Pool> &p;
        Swap(ckks_ctx &cc, std::unique_ptr<Pool> &pp) : c(cc), p(pp) { c.pool.swap(p); }
        ~Swap() { c.pool.swap(p); }
    } swap_(c, other);
    Ct r = mul(c, a, b);
    GCK_HIP(hipMemcpyAsync(out.data.ptr, r->data.ptr, r->data.words * 8, hipMemcpyDeviceToDevice, c.stream));
    out.scale = r->scale;
}

}  // namespace gck
