// Batched CMB log-likelihood without any device allocation, for callers that
// cannot allocate (code under HIP graph capture, tight serving loops): the
// only device memory the one-kernel BF16 / split-BF16 path needs beyond the
// caller's theta and logL (the emulator's model vector, or, for the
// one-network models whose chi^2 runs in the emulator's epilogue, its tile
// partials) lives in a file-scope device array of SCRATCH_BYTES per GPU
// instead of the model's grow-on-demand workspace.
//
// The array's address on each device is taken once, with that device current,
// when the first model is created on it (hipGetSymbolAddress); host code only
// ever passes that address, never the array's name.  Every call on a GPU
// shares the array: calls that overlap in time on one GPU race, and a call
// leaves its model vectors there (every row a call reads, it wrote first, so
// nothing needs clearing).
#include <mutex>

#include "devutil.h"
#include "nsmi.h"

namespace nsmi {

constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;     // 64 MiB per GPU

static __device__ __align__(256) float scratch[SCRATCH_BYTES / sizeof(float)];

constexpr int MAX_DEVICES = 64;
static void* g_scratch_ptr[MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

void scratch_init(int device) {
    NS_CHECK(device >= 0 && device < MAX_DEVICES, NS_E_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    void* p = nullptr;
    NS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));      // the caller made `device` current
    NS_CHECK(p != nullptr, NS_E_HIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[device] = p;
}

size_t scratch_bytes() { return SCRATCH_BYTES; }

void loglike_batch_noalloc(ns_model* m, const double* theta, int64_t ld, int64_t B, double* logl, int prec,
                           hipStream_t s) {
    const bool cmb = m->kind == NS_MODEL_CMB_DIAG || m->kind == NS_MODEL_CMB_BLOCK || m->kind == NS_MODEL_CMB_CV;
    NS_CHECK(cmb, NS_E_UNSUPPORTED, "the allocation-free likelihood covers the CMB model kinds");
    // FP64 on a narrow diagonal model: emulator and chi^2 in one kernel, no scratch at all
    if (prec == NS_FP64) {
        NS_CHECK(m->kind == NS_MODEL_CMB_DIAG && m->nets[0]->narrow64, NS_E_UNSUPPORTED,
                 "the allocation-free FP64 form covers the one-kernel narrow diagonal model only");
        if (B == 0) return;
        m->noalloc_call = true;
        const bool ok = emulator_forward_f64_narrow(m, theta, ld, B, nullptr, 0, m->spec_log[0], logl, nullptr, s);
        m->noalloc_call = false;
        NS_CHECK(ok, NS_E_UNSUPPORTED, "the one-kernel FP64 forward is switched off (NSMI_NO_FUSED_MLP)");
        return;
    }
    NS_CHECK(prec == NS_BF16 || prec == NS_BF16X3, NS_E_UNSUPPORTED,
             "the allocation-free likelihood runs the one-kernel BF16 and split-BF16 forms (and narrow FP64)");
    for (const Net* net : m->nets)
        NS_CHECK(net->fused, NS_E_UNSUPPORTED, "the allocation-free likelihood needs one-kernel emulator networks");
    const int64_t n = cmb_row_stride(m), sp = cmb_spec_stride(m);
    const size_t per_row = (size_t)n * sizeof(float);
    const int64_t max_rows = (int64_t)(SCRATCH_BYTES / per_row);
    NS_CHECK(B <= max_rows, NS_E_SHAPE,
             "batch of " + std::to_string(B) + " walkers needs " + std::to_string((size_t)B * per_row) +
                 " bytes of scratch; the allocation-free likelihood holds " + std::to_string(SCRATCH_BYTES) +
                 " bytes per GPU (at most " + std::to_string(max_rows) + " walkers for this model)");
    if (B == 0) return;
    NS_CHECK(m->device >= 0 && m->device < MAX_DEVICES && g_scratch_ptr[m->device], NS_E_HIP,
             "scratch array not set up on this device");
    char* base = static_cast<char*>(g_scratch_ptr[m->device]);
    const int G = (int)m->nets.size();
    int ids[4];
    void* outs[4];
    for (int g = 0; g < G; ++g) {
        ids[g] = g;
        outs[g] = base + (size_t)g * sp * sizeof(float);
    }
    static const int raw[4] = {0, 0, 0, 0};
    m->noalloc_call = true;
    try {
        // the same launches as ns_loglike_batch: chi^2 in the epilogue where it applies
        if (chi2_fused_part_bytes(m, B) <= SCRATCH_BYTES &&
            emulator_chi2_fused(m, theta, ld, B, logl, prec, nullptr, s, reinterpret_cast<double*>(base))) {
            m->noalloc_call = false;
            return;
        }
        const bool ok = emulator_forward_fused(m, ids, G, theta, ld, B, outs, n,
                                               m->kind == NS_MODEL_CMB_CV ? raw : m->spec_log.data(), prec, nullptr,
                                               s);
        NS_CHECK(ok, NS_E_UNSUPPORTED, "one-kernel emulator unavailable for this model and form");
        cmb_chi2(m, theta, ld, B, base, logl, prec, nullptr, s);
    } catch (...) {
        m->noalloc_call = false;
        throw;
    }
    m->noalloc_call = false;
}

}  // namespace nsmi
