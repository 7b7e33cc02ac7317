// Diagnostic entry points: read back what a plan holds on the device.
#include <cmath>
#include <cstring>
#include <vector>

#include "zm_internal.h"

namespace {

float bf16_value(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, sizeof f);
    return f;
}

// IEEE binary16 -> float (exact).
float half_value(uint16_t h) {
    const int s = h >> 15, e = (h >> 10) & 31, f = h & 1023;
    float v;
    if (e == 0)
        v = std::ldexp((float)f, -24);
    else if (e == 31)
        v = f ? NAN : INFINITY;
    else
        v = std::ldexp((float)(1024 + f), e - 25);
    return s ? -v : v;
}

}  // namespace

using namespace zm;

extern "C" {

zm_status zm_operand_table(zm_plan_t p, double* host_out, size_t n_elems) {
    if (!p || !host_out) return fail(ZM_EINVAL, "null plan or output");
    if (!p->d_thi) return fail(ZM_EUNSUPPORTED, "the plan holds no projection operand (n_max beyond the moment kernels)");
    const size_t need = (size_t)p->num_moments * p->R;
    if (n_elems < need) return fail(ZM_EINVAL, "output too small: need num_moments * rings elements");
    ZM_DEVICE(p->device);
    const size_t n = (size_t)p->table_rows * p->Rp;
    const bool split = p->dtype == ZM_BF16X2 || p->dtype == ZM_F16X2;
    const size_t esz = p->dtype == ZM_F64 ? 8 : (p->dtype == ZM_F32 ? 4 : 2);
    std::vector<unsigned char> hi(n * esz), lo(split ? n * esz : 0);
    std::vector<float> scale(p->dtype == ZM_F16X2 ? p->table_rows : 0);
    ZM_HIP(hipMemcpy(hi.data(), p->d_thi, hi.size(), hipMemcpyDeviceToHost));
    if (split) ZM_HIP(hipMemcpy(lo.data(), p->d_tlo, lo.size(), hipMemcpyDeviceToHost));
    if (!scale.empty())
        ZM_HIP(hipMemcpy(scale.data(), p->d_rowscale, scale.size() * sizeof(float), hipMemcpyDeviceToHost));
    const int g = (p->dtype == ZM_F64 || p->dtype == ZM_F32) ? 4 : 8;
    for (int nn = 0; nn <= p->n_max; ++nn)
        for (int m = nn & 1; m <= nn; m += 2) {
            const int row = p->blk_toff[m] + (nn - m) / 2;
            double* o = host_out + (size_t)canon_index(nn, m) * p->R;
            for (int r = 0; r < p->R; ++r) {
                const size_t k = op_index(row, r, p->Rp, g);
                double v = 0.0;
                switch (p->dtype) {
                    case ZM_F64: std::memcpy(&v, &hi[8 * k], 8); break;
                    case ZM_F32: {
                        float f;
                        std::memcpy(&f, &hi[4 * k], 4);
                        v = f;
                        break;
                    }
                    case ZM_BF16X2: {
                        uint16_t a, b;
                        std::memcpy(&a, &hi[2 * k], 2);
                        std::memcpy(&b, &lo[2 * k], 2);
                        v = (double)bf16_value(a) + (double)bf16_value(b);
                        break;
                    }
                    default: {
                        uint16_t a, b;
                        std::memcpy(&a, &hi[2 * k], 2);
                        std::memcpy(&b, &lo[2 * k], 2);
                        v = ((double)half_value(a) + (double)half_value(b)) * (double)scale[row];
                        break;
                    }
                }
                o[r] = v;
            }
        }
    return ZM_OK;
}

}  // extern "C"
