// White-box check of the work split of the batched scans (a GPU test runs it; it links libbl.so and calls
// the library's internal launchers).  The FP64 matrix-core scan (modes 0-2, every variant) is compared with
// dot products in FP64 on the CPU for sampled columns, to 1e-12 of sum_i |x_ij b_ib|; the BF16 scan (two and
// three pieces) with the FP64 scan, to the stated BF16 bound.  List lengths cover one column, lists shorter
// than one tile per workgroup (every tile cut by rows), and lists that give each workgroup whole tiles and
// leave some to cut, with the length on the host and on the device.  Every run is repeated (the results
// must be equal bit for bit) and the entries outside the list must be left untouched.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "bl.h"
#include "internal.h"
using namespace blk;

#define CK(x)                                                                                   \
    do {                                                                                        \
        hipError_t e_ = (x);                                                                    \
        if (e_ != hipSuccess) {                                                                 \
            printf("HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__);             \
            exit(2);                                                                            \
        }                                                                                       \
    } while (0)

int main() {
    const int64_t n = 1037, p = 140000;   // a ragged last chunk of 13 rows
    const int nprob = 61;
    const int64_t n_pad = batch_pad(n);
    std::mt19937_64 rng(20240611);
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<float> X((size_t)n * p);
    for (auto& v : X) v = (float)nd(rng);
    std::vector<double> B((size_t)n_pad * BNP, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int b = 0; b < nprob; ++b) B[i * BNP + b] = nd(rng) * (1 + b % 5);
    std::vector<BatchScalars> bs(BNP);
    for (int b = 0; b < BNP; ++b) {
        memset(&bs[b], 0, sizeof(BatchScalars));
        double sr = 0, rss = 0;
        for (int64_t i = 0; i < n; ++i) {
            sr += B[i * BNP + b];
            rss += B[i * BNP + b] * B[i * BNP + b];
        }
        bs[b].sum_r = sr;
        bs[b].rss = rss;
        bs[b].n_rows = n - (b % 7);
    }
    std::vector<double> c((size_t)BNP * p), s((size_t)BNP * p);
    for (auto& v : c) v = 0.01 * nd(rng);
    for (auto& v : s) v = 0.5 + std::fabs(nd(rng));
    std::vector<int32_t> perm(p);
    for (int64_t j = 0; j < p; ++j) perm[j] = (int32_t)j;
    std::shuffle(perm.begin(), perm.end(), rng);
    std::vector<int64_t> samp;   // sampled list positions
    for (int64_t t = 0; t < p; ++t)
        if (t < 200 || t % 331 == 0 || t >= p - 40) samp.push_back(t);

    float* dX;
    double *dB, *dc, *ds, *dout, *dout2, *dz64, *dpart, *dbfpart;
    BatchScalars* dbs;
    int32_t* dcols;
    int64_t* dlen;
    __bf16* dRp;
    const size_t OUT = (size_t)BNP * p * 8;
    CK(hipMalloc(&dX, X.size() * 4));
    CK(hipMalloc(&dB, B.size() * 8));
    CK(hipMalloc(&dc, c.size() * 8));
    CK(hipMalloc(&ds, s.size() * 8));
    CK(hipMalloc(&dout, OUT));
    CK(hipMalloc(&dout2, OUT));
    CK(hipMalloc(&dz64, OUT));
    CK(hipMalloc(&dpart, bscan_part_bytes()));
    CK(hipMalloc(&dbfpart, std::max(bscan_bf16_part_bytes(2), bscan_bf16_part_bytes(3))));
    CK(hipMalloc(&dbs, BNP * sizeof(BatchScalars)));
    CK(hipMalloc(&dcols, p * 4));
    CK(hipMalloc(&dlen, 8));
    CK(hipMalloc(&dRp, bscan_bf16_pieces_bytes(n, 3)));
    CK(hipMemcpy(dX, X.data(), X.size() * 4, hipMemcpyHostToDevice));
    CK(hipMemcpy(dB, B.data(), B.size() * 8, hipMemcpyHostToDevice));
    CK(hipMemcpy(dc, c.data(), c.size() * 8, hipMemcpyHostToDevice));
    CK(hipMemcpy(ds, s.data(), s.size() * 8, hipMemcpyHostToDevice));
    CK(hipMemcpy(dbs, bs.data(), BNP * sizeof(BatchScalars), hipMemcpyHostToDevice));
    CK(hipMemcpy(dcols, perm.data(), p * 4, hipMemcpyHostToDevice));
    const Mat mt{dX, BL_X_F32, n, p, n, nullptr};
    const int64_t lens[] = {1, 129, 20000, 70000, p};
    std::vector<double> o((size_t)BNP * p), o2((size_t)BNP * p), z64((size_t)BNP * p);
    int failures = 0;

    // the listed positions, untouched entries and repeat check of one run pair (sentinel: all bits set, NaN)
    auto check_layout = [&](int64_t len, const char* what) -> bool {
        CK(hipMemcpy(o.data(), dout, OUT, hipMemcpyDeviceToHost));
        CK(hipMemcpy(o2.data(), dout2, OUT, hipMemcpyDeviceToHost));
        int64_t nnd = 0, nunw = 0, nover = 0;
        if (memcmp(o.data(), o2.data(), OUT) != 0) nnd = 1;
        std::vector<char> listed(p, 0);
        for (int64_t t = 0; t < len; ++t) listed[perm[t]] = 1;
        for (int b = 0; b < nprob; ++b)
            for (int64_t j = 0; j < p; j += 5) {
                const double v = o[(size_t)b * p + j];
                if (listed[j] && std::isnan(v)) ++nunw;
                if (!listed[j] && !std::isnan(v)) ++nover;
            }
        if (nnd || nunw || nover) {
            printf("FAIL %s len %ld: repeat differs %ld, unwritten %ld, written outside the list %ld\n", what,
                   (long)len, (long)nnd, (long)nunw, (long)nover);
            return false;
        }
        return true;
    };

    // FP64 matrix-core scan, modes 0-2, every variant, against the CPU
    for (int mode = 0; mode < 3; ++mode) {
        std::vector<double> ref(samp.size() * nprob), mag(samp.size() * nprob);
        for (size_t k = 0; k < samp.size(); ++k) {
            const int64_t j = perm[samp[k]];
            for (int b = 0; b < nprob; ++b) {
                double a = 0, am = 0;
                for (int64_t i = 0; i < n; ++i) {
                    double x = (double)X[j * n + i];
                    if (mode == 1) x = x * x;
                    a += x * B[i * BNP + b];
                    am += std::fabs(x * B[i * BNP + b]);
                }
                const size_t bj = (size_t)b * p + j;
                if (mode == 2) {
                    const double den = (double)bs[b].n_rows * s[bj];
                    a = (a - c[bj] * bs[b].sum_r) / den;
                    am = (am + std::fabs(c[bj] * bs[b].sum_r)) / den;
                }
                ref[k * nprob + b] = a;
                mag[k * nprob + b] = am;
            }
        }
        for (int variant = 0; variant < 6; ++variant) {
            double worst = 0;
            for (int64_t len : lens)
                for (int dev = 0; dev < 2; ++dev) {
                    CK(hipMemcpy(dlen, &len, 8, hipMemcpyHostToDevice));
                    CK(hipMemset(dout, 0xFF, OUT));
                    CK(launch_bscan(mt, mode, dcols, dev ? dlen : nullptr, len, dB, nprob, dbs, dc, ds, nullptr, dpart,
                                    dout, 0, variant));
                    CK(hipMemcpy(dout2, dout, OUT, hipMemcpyDeviceToDevice));
                    CK(launch_bscan(mt, mode, dcols, dev ? dlen : nullptr, len, dB, nprob, dbs, dc, ds, nullptr, dpart,
                                    dout2, 0, variant));
                    CK(hipDeviceSynchronize());
                    char what[64];
                    snprintf(what, sizeof what, "fp64 mode %d variant %d dev %d", mode, variant, dev);
                    if (!check_layout(len, what)) {
                        ++failures;
                        continue;
                    }
                    int64_t nbad = 0;
                    for (size_t k = 0; k < samp.size(); ++k) {
                        if (samp[k] >= len) continue;
                        const int64_t j = perm[samp[k]];
                        for (int b = 0; b < nprob; ++b) {
                            const double d = std::fabs(o[(size_t)b * p + j] - ref[k * nprob + b]);
                            const double tol = 1e-12 * mag[k * nprob + b];
                            worst = std::max(worst, d / tol);
                            if (!(d <= tol)) ++nbad;
                        }
                    }
                    if (nbad) {
                        printf("FAIL %s len %ld: %ld sampled values off the FP64 reference\n", what, (long)len,
                               (long)nbad);
                        ++failures;
                    }
                }
            printf("fp64 scan mode %d variant %d: largest difference %.2e of the tolerance\n", mode, variant, worst);
            fflush(stdout);
        }
    }

    // BF16 scan (two and three pieces) against the FP64 scan, to the BF16 bound
    for (int pc = 2; pc <= 3; ++pc) {
        const double rel = bscan_bf16_rel(n, pc);
        CK(launch_b_r_pieces(dB, n, nprob, pc, dRp, 0));
        double worst = 0;
        for (int64_t len : lens)
            for (int dev = 0; dev < 2; ++dev) {
                CK(hipMemcpy(dlen, &len, 8, hipMemcpyHostToDevice));
                CK(launch_bscan(mt, 2, dcols, nullptr, len, dB, nprob, dbs, dc, ds, nullptr, dpart, dz64, 0, 1));
                CK(hipMemset(dout, 0xFF, OUT));
                CK(launch_bscan_bf16(mt, dcols, dev ? dlen : nullptr, len, pc, dRp, nprob, dbs, dc, ds, nullptr,
                                     dbfpart, dout, 0));
                CK(hipMemcpy(dout2, dout, OUT, hipMemcpyDeviceToDevice));
                CK(launch_bscan_bf16(mt, dcols, dev ? dlen : nullptr, len, pc, dRp, nprob, dbs, dc, ds, nullptr,
                                     dbfpart, dout2, 0));
                CK(hipDeviceSynchronize());
                char what[64];
                snprintf(what, sizeof what, "bf16 pieces %d dev %d", pc, dev);
                if (!check_layout(len, what)) {
                    ++failures;
                    continue;
                }
                CK(hipMemcpy(z64.data(), dz64, OUT, hipMemcpyDeviceToHost));
                int64_t nbad = 0;
                for (int64_t t = 0; t < len; t += (len > 5000 ? 7 : 1)) {
                    const int64_t j = perm[t];
                    for (int b = 0; b < nprob; ++b) {
                        const size_t bj = (size_t)b * p + j;
                        const double nb = (double)bs[b].n_rows;
                        const double err = rel * std::sqrt(nb * (s[bj] * s[bj] + c[bj] * c[bj])) * std::sqrt(bs[b].rss) /
                                               (nb * s[bj]) + 1e-14 * std::fabs(z64[bj]);
                        const double d = std::fabs(o[bj] - z64[bj]);
                        worst = std::max(worst, d / err);
                        if (!(d <= err)) ++nbad;
                    }
                }
                if (nbad) {
                    printf("FAIL %s len %ld: %ld values outside the BF16 bound\n", what, (long)len, (long)nbad);
                    ++failures;
                }
            }
        printf("bf16 scan, %d pieces: largest difference %.2e of the bound\n", pc, worst);
        fflush(stdout);
    }
    printf(failures ? "FAILED %d\n" : "OK\n", failures);
    return failures ? 1 : 0;
}
