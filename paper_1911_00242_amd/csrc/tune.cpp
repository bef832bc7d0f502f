// Measurements behind the choice of arithmetic form per mixed-precision product: the error
// of each form on seeded operands of the product's shape against the FP64 MFMA kernel,
// and a small on-disk cache of measurements keyed by device and product shape.
#include "tune.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <random>
#include <sstream>
#include <vector>

#include "mixed.h"

namespace ck {

namespace {

// Dense tables for A [1][M][K], B [1][N][K], C [1][M][N] (element offsets).
std::vector<int64_t> dense_tables(int M, int N, int K, size_t off[5]) {
    std::vector<int64_t> t;
    off[0] = t.size();
    for (int m = 0; m < M; ++m) t.push_back((int64_t)m * K);
    off[1] = t.size();
    for (int k = 0; k < K; ++k) t.push_back(k);
    off[2] = t.size();
    for (int n = 0; n < N; ++n) t.push_back((int64_t)n * K);
    off[3] = t.size();
    for (int m = 0; m < M; ++m) t.push_back((int64_t)m * N);
    off[4] = t.size();
    for (int n = 0; n < N; ++n) t.push_back(n);
    return t;
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

std::vector<double> form_errors(int M, int N, int K, uint64_t seed, hipStream_t st) {
    // operands: complex numbers with independent standard normal parts; the error of a
    // form is max |C_form - C_fp64| / max |C_fp64|
    const int64_t na = (int64_t)M * K, nb = (int64_t)N * K, nc = (int64_t)M * N;
    std::mt19937_64 rng(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<double> ha(2 * na), hb(2 * nb);
    for (auto &x : ha) x = nd(rng);
    for (auto &x : hb) x = nd(rng);
    size_t off[5];
    std::vector<int64_t> tab = dense_tables(M, N, K, off);
    const int64_t pa = (na + 63) / 64 * 64, pb = (nb + 63) / 64 * 64;
    DevBuf dA, dB, dC, dR, dT, dZ, sA, sB;
    CK_CHECK(hipMalloc(&dA.p, std::max<int64_t>(na, 1) * sizeof(cd)));
    CK_CHECK(hipMalloc(&dB.p, std::max<int64_t>(nb, 1) * sizeof(cd)));
    CK_CHECK(hipMalloc(&dC.p, nc * sizeof(cd)));
    CK_CHECK(hipMalloc(&dR.p, nc * sizeof(cd)));
    CK_CHECK(hipMalloc(&dT.p, tab.size() * sizeof(int64_t)));
    CK_CHECK(hipMalloc(&dZ.p, 256));
    CK_CHECK(hipMalloc(&sA.p, 8 * pa));
    CK_CHECK(hipMalloc(&sB.p, 8 * pb));
    CK_CHECK(hipMemcpyAsync(dA.p, ha.data(), na * sizeof(cd), hipMemcpyHostToDevice, st));
    CK_CHECK(hipMemcpyAsync(dB.p, hb.data(), nb * sizeof(cd), hipMemcpyHostToDevice, st));
    CK_CHECK(hipMemcpyAsync(dT.p, tab.data(), tab.size() * sizeof(int64_t), hipMemcpyHostToDevice, st));
    CK_CHECK(hipMemsetAsync(dZ.p, 0, 256, st));
    const int64_t *T = (const int64_t *)dT.p;
    GemmOps<cd> op{};
    op.A = (const cd *)dA.p; op.B = (const cd *)dB.p; op.C = (cd *)dR.p; op.zeros = (const cd *)dZ.p;
    op.a_row = T + off[0]; op.a_k = T + off[1]; op.b_col = T + off[2]; op.b_k = T + off[1];
    op.c_row = T + off[3]; op.c_col = T + off[4];
    op.G = 1; op.M = M; op.N = N; op.K = K; op.alpha = 1.0; op.beta = 0.0;
    gemm_f64(op, st);
    std::vector<double> ref(2 * nc), got(2 * nc);
    CK_CHECK(hipMemcpyAsync(ref.data(), dR.p, nc * sizeof(cd), hipMemcpyDeviceToHost, st));
    CK_CHECK(hipStreamSynchronize(st));
    double scale = 0.0;
    for (int64_t e = 0; e < nc; ++e) scale = std::max(scale, std::hypot(ref[2 * e], ref[2 * e + 1]));
    std::vector<double> err(ARITH_COUNT, 0.0);
    for (int f = 0; f < ARITH_COUNT; ++f) {
        SplitOps so{};
        so.C = (cd *)dC.p; so.Cs = nullptr; so.zeros = (const uint16_t *)dZ.p;
        so.a_row = op.a_row; so.a_k = op.a_k; so.b_col = op.b_col; so.b_k = op.b_k;
        so.c_row = op.c_row; so.c_col = op.c_col; so.cs_row = so.cs_col = nullptr;
        so.G = 1; so.M = M; so.N = N; so.K = K; so.alpha = 1.0; so.beta = 0.0;
        so.fast = (K % 8 == 0) ? 1 : 0;
        so.A = (const uint16_t *)sA.p;
        so.B = (const uint16_t *)sB.p;
        if (arith_c64(f)) {
            launch_to_c64(na, (const cd *)dA.p, (cf *)sA.p, st);
            launch_to_c64(nb, (const cd *)dB.p, (cf *)sB.p, st);
            gemm_c64(so, f, st);
        } else {
            launch_split(na, (const cd *)dA.p, (uint16_t *)sA.p, st);
            launch_split(nb, (const cd *)dB.p, (uint16_t *)sB.p, st);
            gemm_split(so, st);
        }
        CK_CHECK(hipMemcpyAsync(got.data(), dC.p, nc * sizeof(cd), hipMemcpyDeviceToHost, st));
        CK_CHECK(hipStreamSynchronize(st));
        double worst = 0.0;
        for (int64_t e = 0; e < nc; ++e)
            worst = std::max(worst, std::hypot(got[2 * e] - ref[2 * e], got[2 * e + 1] - ref[2 * e + 1]));
        err[f] = scale > 0.0 ? worst / scale : worst;
    }
    return err;
}

std::string device_key() {
    int dev = 0;
    hipDeviceProp_t p{};
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string name = std::string(p.name) + "/" + p.gcnArchName;
    for (char &c : name)
        if (c == ' ' || c == '|' || c == '\n') c = '_';
    return name;
}

std::string tune_key(const std::string &dev, int G, int M, int N, int K, int fast) {
    std::ostringstream s;
    s << dev << "|" << G << "," << M << "," << N << "," << K << "," << fast;
    return s.str();
}

bool cache_lookup(const char *path, const std::string &key, TuneRecord &out) {
    if (!path) return false;
    std::ifstream in(path);
    std::string line;
    bool found = false;
    while (std::getline(in, line)) {  // the last record of a key wins
        std::istringstream s(line);
        std::string k;
        TuneRecord r;
        if (!(s >> k) || k != key) continue;
        bool ok = true;
        for (int f = 0; f < ARITH_COUNT && ok; ++f) ok = static_cast<bool>(s >> r.ms[f]);
        for (int f = 0; f < ARITH_COUNT && ok; ++f) ok = static_cast<bool>(s >> r.err[f]);
        if (ok) {
            out = r;
            found = true;
        }
    }
    return found;
}

void cache_store(const char *path, const std::string &key, const TuneRecord &r) {
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;  // a read-only cache location only costs a re-measurement next time
    std::fprintf(f, "%s", key.c_str());
    for (int i = 0; i < ARITH_COUNT; ++i) std::fprintf(f, " %.6g", r.ms[i]);
    for (int i = 0; i < ARITH_COUNT; ++i) std::fprintf(f, " %.6g", r.err[i]);
    std::fprintf(f, "\n");
    std::fclose(f);
}

}  // namespace ck
