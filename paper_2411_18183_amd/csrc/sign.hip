// Signature of every key (Section 3.1), and the plain full-key hash of the
// baseline simple hash join (Section 2), on gfx950.  The per-window work
// decomposition and the GF(2^16) chunk arithmetic are in sign_window.h.
#include "sign_window.h"

namespace {

// 16 waves per block: one LDS copy of the GF tables (35 KB) serves twice as
// many waves, so two blocks (32 waves) fit a CU instead of three blocks of 8.
constexpr int kBlock = 1024;
constexpr int kWaves = kBlock / ASJ_WAVE;
// Grid, when the kernel sizes the windows: this many rounds of the blocks
// the device holds at once, each block looping over windows.  Measured on
// 32k to 1.3M keys of 64 B to 5.5 KB: one round balanced long keys poorly
// (DNA keys 10% slower); four and eight rounds came within 2% of each
// other on every set but 1M keys of 64 bytes (eight: 7%, 1.5 us slower)
// and 1M DNA keys (eight: 2% faster), and the batch whose blocks also
// wrote the slot fill and window maps (256 joins, 6.3M build keys) signed
// 6% slower on four rounds than on eight.
constexpr int kSignRounds = 8;

// out[k * stride] = signature of key k (its low word with four GF(2^16)
// components, whose high word goes to out_hi[k * stride]).  With has_prep
// the blocks first do their part of a batch's preparation.  A wave signs
// windows of kpw consecutive keys (1 .. 64, or 0: chosen here from the
// keys' mean length by asj_auto_kpw): long keys fill a window's passes with
// few keys, and fewer keys per window give few long keys enough windows to
// occupy every compute unit.
template <int MODE, int NSYM>
__global__ __launch_bounds__(kBlock) void sign_kernel(const uint8_t *__restrict__ data,
                                                      const int64_t *__restrict__ off, int64_t n,
                                                      uint32_t *__restrict__ out, uint32_t *__restrict__ out_hi,
                                                      int stride, const uint16_t *__restrict__ gtab,
                                                      const int32_t *__restrict__ status, asj_batch_prep prep,
                                                      int has_prep, int kpw)
{
    constexpr bool kHi = MODE == ASJ_MODE_SIG16 && NSYM == 4;
    if (has_prep) asj_batch_prep_run(prep, blockIdx.x, gridDim.x, threadIdx.x, kBlock);
    if (status && *status != 0) return; // the inputs failed validation: read no key (same for every thread)
    const int64_t end = off[n]; // the keys' bytes end here
    const int64_t bytes = end - off[0]; // both loads in flight while the tables load
    // kpw = 0: the grid was sized for the smallest windows.  Blocks that
    // have a window whatever the size (windows of 64 keys cover them) load
    // the GF tables at once; the others first read the keys' extent and
    // leave if the chosen windows do not reach them.
    if (kpw <= 0 && (int64_t)blockIdx.x * kWaves * ASJ_WAVE >= n) { // block-uniform
        kpw = asj_auto_kpw(n, bytes);
        if ((int64_t)blockIdx.x * kWaves * kpw >= n) return;
    }
    __shared__ uint16_t tab[asj::TabWords<MODE>::value];
    __shared__ int64_t kst[kWaves][ASJ_WAVE];
    __shared__ int32_t kex[kWaves][ASJ_WAVE];
    __shared__ uint32_t kacc[kWaves][ASJ_WAVE];
    __shared__ int32_t kown[kWaves][ASJ_WAVE];
    __shared__ uint32_t kacc2[kHi ? kWaves : 1][ASJ_WAVE];
    asj::load_tables<MODE, kBlock>(tab, gtab);

    const int wave = threadIdx.x / ASJ_WAVE;
    const int lane = threadIdx.x % ASJ_WAVE;
    if (kpw <= 0) kpw = asj_auto_kpw(n, bytes);
    const int64_t nwin = (n + kpw - 1) / kpw;
    for (int64_t w = (int64_t)blockIdx.x * kWaves + wave; w < nwin; w += (int64_t)gridDim.x * kWaves) {
        const int64_t k = w * kpw + lane;
        const bool mine = lane < kpw && k < n;
        int64_t s = 0;
        int len = 0;
        if (mine) {
            s = off[k];
            len = (int)(off[k + 1] - s);
        }
        uint32_t hi = 0;
        const uint32_t v = asj::sign_window<MODE, NSYM>(data, s, len, end, kst[wave], kex[wave], kacc[wave], kown[wave], tab,
                                                        gtab, kacc2[kHi ? wave : 0], hi);
        if (mine) {
            out[k * stride] = v;
            if (kHi) out_hi[k * stride] = hi;
        }
    }
}

template <int MODE, int NSYM>
hipError_t launch(const asj_keys *k, uint32_t *out, uint32_t *out_hi, int stride, const uint16_t *tab, int grid_cap,
                  const int32_t *status, const asj_batch_prep *prep, int kpw, hipStream_t st)
{
    const asj_batch_prep none = {};
    const int kmin = kpw > 0 ? kpw : asj_kpw_min(k->n); // 0: the kernel picks asj_kpw_min .. 64
    const int64_t nwin = (k->n + kmin - 1) / kmin;
    int64_t blocks = (nwin + kWaves - 1) / kWaves;
    if (blocks > grid_cap) blocks = grid_cap;
    if (kpw <= 0) {
        static const int64_t resident =
            asj_resident_blocks(reinterpret_cast<const void *>(&sign_kernel<MODE, NSYM>), kBlock);
        if (resident > 0 && blocks > resident * kSignRounds) blocks = resident * kSignRounds;
    }
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((sign_kernel<MODE, NSYM>), dim3((unsigned)blocks), dim3(kBlock), 0, st, k->data, k->offsets,
                       k->n, out, out_hi, stride, tab, status, prep ? *prep : none, prep ? 1 : 0, kpw);
    return hipGetLastError();
}

} // namespace

hipError_t asj_launch_sign(int mode, int nsym, const asj_keys *k, uint32_t *out, const uint16_t *tab, int grid_cap,
                           hipStream_t st, const int32_t *status, uint32_t *out_hi, int stride,
                           const asj_batch_prep *prep, int kpw)
{
    if (k->n == 0) return prep ? asj_launch_batch_prep(prep, st) : hipSuccess;
    if (stride < 1) return hipErrorInvalidValue;
    if (kpw < 0 || kpw > ASJ_WAVE) kpw = ASJ_WAVE; // 0: chosen by the kernel
    if (mode == ASJ_MODE_SIG16 && nsym == 4) {
        if (!out_hi) return hipErrorInvalidValue;
        return launch<ASJ_MODE_SIG16, 4>(k, out, out_hi, stride, tab, grid_cap, status, prep, kpw, st);
    }
    if (mode == ASJ_MODE_SIG16 && nsym == 2)
        return launch<ASJ_MODE_SIG16, 2>(k, out, nullptr, stride, tab, grid_cap, status, prep, kpw, st);
    if (mode == ASJ_MODE_SIG16 && nsym == 1)
        return launch<ASJ_MODE_SIG16, 1>(k, out, nullptr, stride, tab, grid_cap, status, prep, kpw, st);
    if (mode == ASJ_MODE_SIG8 && nsym == 4)
        return launch<ASJ_MODE_SIG8, 4>(k, out, nullptr, stride, tab, grid_cap, status, prep, kpw, st);
    if (mode == ASJ_MODE_SIG8 && nsym == 2)
        return launch<ASJ_MODE_SIG8, 2>(k, out, nullptr, stride, tab, grid_cap, status, prep, kpw, st);
    if (mode == ASJ_MODE_PLAIN) return launch<ASJ_MODE_PLAIN, 1>(k, out, nullptr, stride, tab, grid_cap, status, prep, kpw, st);
    return hipErrorInvalidValue;
}
