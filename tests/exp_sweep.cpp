// Sweep of the device exp's fast path on the host: wherever it does not flag a hard case,
// its result equals the double-double path's; for ordinary arguments the bare core gives the
// fast path's result and flag.  Every `stride`-th binary32 argument in
// [underflow threshold, overflow threshold); stride 1 is the exhaustive sweep.
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>
#define SG_HD inline
#include "../paper_1410_6685_amd/csrc/sg_exp.h"

int main(int argc, char** argv) {
    const uint64_t stride = argc > 1 ? std::strtoull(argv[1], nullptr, 10) : 1;
    const int nt = argc > 2 ? std::atoi(argv[2]) : 8;
    const uint64_t npos = SG_EXP_OVF_BITS, nneg = SG_EXP_UNF_BITS - 0x80000000u + 1;
    std::atomic<uint64_t> bad{0}, hard{0}, total{0};
    std::vector<std::thread> th;
    for (int w = 0; w < nt; ++w)
        th.emplace_back([&, w]() {
            uint64_t b = 0, h = 0, n = 0;
            for (uint64_t u = (uint64_t)w * stride; u < npos + nneg; u += (uint64_t)nt * stride) {
                const uint32_t bits = u < npos ? (uint32_t)u : (uint32_t)(0x80000000u + (u - npos));
                const float t = sgx::u2f(bits);
                bool hd;
                const float f = sgx::exp_rn_fast(t, SG_EXPF_TAB, hd);
                ++n;
                if (sgx::exp_ordinary(t)) {
                    bool hc;
                    const float fc = sgx::exp_rn_core(t, SG_EXPF_TAB, hc);
                    if (hc != hd || (!hd && sgx::f2u(fc) != sgx::f2u(f))) {
                        if (b < 5) std::printf("core differs t=%a\n", t);
                        ++b;
                    }
                }
                if (hd) { ++h; continue; }
                if (sgx::f2u(f) != sgx::f2u(sgx::exp_rn_slow(t))) {
                    if (b < 5) std::printf("mismatch t=%a fast=%a\n", t, f);
                    ++b;
                }
            }
            bad += b;
            hard += h;
            total += n;
        });
    for (auto& t : th) t.join();
    std::printf("total %llu hard %llu bad %llu\n", (unsigned long long)total, (unsigned long long)hard,
                (unsigned long long)bad);
    return bad != 0;
}
