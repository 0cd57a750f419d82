// Construction of the GF(2^f) constant tables used by the signature kernels
// (Section 3.1: arithmetic in GF(2^f); addition is XOR, every non-zero
// element is a power of the primitive element alpha).
//
// One launch per device at library initialisation.  Every entry is computed
// independently by shift-and-add multiplication with reduction, so the
// kernel needs no sequential table walk.
#include "asj_internal.h"

namespace {

constexpr uint32_t kPoly16 = 0x1100Bu; // x^16 + x^12 + x^3 + x + 1
constexpr uint32_t kPoly8 = 0x11Du;    // x^8 + x^4 + x^3 + x^2 + 1

__device__ uint32_t gf_mul(uint32_t a, uint32_t b, int f, uint32_t poly)
{
    uint32_t r = 0;
    for (int i = 0; i < f; i++) {
        if ((b >> i) & 1u) r ^= a;
        a <<= 1;
        if (a >> f) a ^= poly;
    }
    return r;
}

__device__ uint32_t gf_alpha_pow(uint64_t e, int f, uint32_t poly)
{
    uint32_t result = 1, base = 2; // alpha = x
    while (e) {
        if (e & 1u) result = gf_mul(result, base, f, poly);
        base = gf_mul(base, base, f, poly);
        e >>= 1;
    }
    return result;
}

// exponent of the constant of GF(2^16) pair `idx` (see asj_internal.h); the
// fold constant x^16 is alpha^16 as well.
__device__ uint64_t pair_exponent(int idx)
{
    if (idx == ASJ_TAB_RED) return 16;
    const int j = 1 + (idx - 1) / 17;
    const int r = (idx - 1) % 17;
    if (r < 8) return 32ull * j * r;
    if (r < 16) return 256ull * j * (r - 8);
    return 2048ull * j;
}

__global__ void tables_kernel(uint16_t *tab)
{
    const int b = threadIdx.x; // 0..255
    const int idx = blockIdx.x;
    if (idx > ASJ_NTAB16) { // device-memory pair h = asj_tab_hi(j, k, d)
        const int h = idx - ASJ_NTAB16 - 1;
        const int j = 1 + h / 49, k = (h % 49) / 7, d = 1 + h % 7;
        const uint32_t c = gf_alpha_pow(2048ull * j * d << (3 * k), 16, kPoly16);
        uint16_t *t = tab + ASJ_TAB_HI_BASE + h * ASJ_TAB_WORDS;
        t[b] = (uint16_t)gf_mul((uint32_t)b, c, 16, kPoly16);
        t[256 + b] = (uint16_t)gf_mul((uint32_t)b << 8, c, 16, kPoly16);
        return;
    }
    if (idx < ASJ_NTAB16) {
        const uint32_t c = gf_alpha_pow(pair_exponent(idx), 16, kPoly16);
        uint16_t *t = tab + idx * ASJ_TAB_WORDS;
        t[b] = (uint16_t)gf_mul((uint32_t)b, c, 16, kPoly16);
        t[256 + b] = (uint16_t)gf_mul((uint32_t)b << 8, c, 16, kPoly16);
        return;
    }
    uint16_t *t8 = tab + ASJ_TAB8_BASE;
    // exp8 over [0, 510)
    for (int e = b; e < 510; e += 256) t8[ASJ_TAB8_EXP + e] = (uint16_t)gf_alpha_pow((uint64_t)(e % 255), 8, kPoly8);
    // log8 by search (255 candidates)
    if (b > 0) {
        uint32_t v = 1;
        for (int e = 0; e < 255; e++) {
            if (v == (uint32_t)b) {
                t8[ASJ_TAB8_LOG + b] = (uint16_t)e;
                break;
            }
            v = gf_mul(v, 2u, 8, kPoly8);
        }
    } else {
        t8[ASJ_TAB8_LOG] = 0;
    }
    for (int k = 1; k <= 3; k++)
        t8[ASJ_TAB8_RED + 256 * (k - 1) + b] = (uint16_t)gf_mul((uint32_t)b, gf_alpha_pow(8ull * k, 8, kPoly8), 8, kPoly8);
}

} // namespace

hipError_t asj_launch_tables(uint16_t *tab, hipStream_t st)
{
    hipLaunchKernelGGL(tables_kernel, dim3(ASJ_NTAB16 + 1 + ASJ_NTAB_HI), dim3(256), 0, st, tab);
    return hipGetLastError();
}
