// Host driver of libccsdk: plan, workspace carving, contraction tables, the residual
// pipeline, the iteration with optional DIIS, and the C ABI declared in include/ccsd_k.h.
//
// The residual follows the T2 equation of Sec. 2 of the paper (eq. ori_EqDouble), with
// one regrouping that is exact: the 1/4 tau<mn||ef> part of W_abef is folded into the
// hole-hole intermediate (which then carries 1/2 tau<mn||ef>), since
//   1/2 sum_ef (1/4 sum_mn tau_mn^ab <mn||ef>) tau_ij^ef
//     = 1/2 sum_mn tau_mn^ab (1/4 sum_ef tau_ij^ef <mn||ef>),
// so the particle-particle ladder contracts only the T1-dressed <ab||ef>.
#include "../../include/ccsd_k.h"

#include <algorithm>
#include <memory>
#include <new>
#include <stdexcept>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.h"
#include "gemm_tiles.h"
#include "mixed.h"
#include "noalloc.h"
#include "pack.h"
#include "terms.h"
#include "tune.h"

namespace {

thread_local std::string g_init_error;

// Largest mesh a context plans: the host momentum table holds N_k^3 entries and the
// contraction tables O(N_k^2 n^2) (N_k = 512: 0.5 GB for the table alone).
constexpr int64_t CK_MAX_NK = 512;

using ck::cd;

enum Stage { ST_PP = 0, ST_HH = 1, ST_WMN = 2, ST_WR = 3, ST_RING = 4, ST_RES = 5, ST_COUNT = 6 };

struct Gemm {
    ck::GemmOps<cd> op;
    int stage;
    size_t tab[6];  // offsets (in int64 units) of a_row, a_k, b_col, b_k, c_row, c_col in the table blob
    // packed products only: partner column, split-output row and column offsets (SIZE_MAX: none)
    size_t cs_row = SIZE_MAX, cs_col = SIZE_MAX;
};

struct System {
    ccsd_k_system desc{};
    ck::Mesh mesh{};
    ck::Dims d{};
    std::vector<int32_t> kc;
    std::vector<int64_t> tables;
    Gemm g[5];
    // device memory (carved from the workspace)
    cd *fock = nullptr, *eri[6] = {};
    cd *amp = nullptr, *res = nullptr;  // [t1 | t2], [r1 | r2]
    cd *tau = nullptr, *tauT = nullptr, *Vt = nullptr, *WT = nullptr, *WR = nullptr, *X = nullptr;
    cd *scr = nullptr, *scrq = nullptr, *P1 = nullptr;
    // rearranged hole-hole grouping (grouping 1, FP64 path): the per-block transpose of t2
    // (B operand of the two hole-hole products) and X-tilde = t2 <mn||ef> (WT layout); the
    // W_mnij buffer WT then holds Y-tilde.  gr: X-tilde, 1/4 X-tilde t2, Y-tilde t2
    cd *t2T = nullptr, *XT = nullptr;
    Gemm gr[3];
    bool rearranged() const { return desc.grouping == CCSD_K_GROUPING_REARRANGED; }
    cd *ovvoT = nullptr;  // static ovvo, ovvv, oovv classes with their last two indices swapped
    cd *ovvvT = nullptr, *oovvT = nullptr;
    // mixed path: the integral classes in complex64 only (eri[] is not kept): the three
    // swapped copies above, oovv and ovvv, oooo and ooov, and <ab||ef> on the blocks that
    // hold its doubly canonical pairs (ka <= kb, ke <= kf: the dblk list of ptab, in order)
    ck::cf *ovvoT_c = nullptr, *ovvv_c = nullptr, *ovvvT_c = nullptr, *oovv_c = nullptr, *oovvT_c = nullptr;
    ck::cf *oooo_c = nullptr, *ooov_c = nullptr, *vvvv_c = nullptr;
    ck::cf *r2c = nullptr;  // mixed path: R2 in complex64 (res then holds R1 only)
    cd *zeros = nullptr;  // 256 zero bytes: load target of out-of-range GEMM operand elements
    ck::FWork fw{};
    double *eo = nullptr, *ev = nullptr, *red = nullptr, *redout = nullptr;
    int32_t *dkc = nullptr;
    int64_t *dtab = nullptr;
    // DIIS history: amplitudes (FP64) and error vectors (FP64; complex64 on the mixed path,
    // whose residual carries about 1e-7 relative error, so the overlaps lose nothing)
    std::vector<cd *> dvec, derr;
    std::vector<ck::cf *> derr32;
    // mixed precision: split-BF16 operands (four bf16 per element) of the five products
    bool mixed = false;
    uint16_t *sp_t2 = nullptr, *sp_WR = nullptr, *sp_oovv = nullptr;
    int64_t pl_t2 = 0;  // element count of the T2-shaped split operands, padded
    // the ladder products run on antisymmetric pairs (pack.hip): canonical pair lists per
    // group (host and device, int32), the packed products and their split operands
    // vlist [N][PV] | olist [N][PO] | vpos [N][N][v][v] | opos [N][N][o][o] | dblk | ablk |
    // vblk [N][N][N] (a block's place in dblk, -1 when it is not there)
    std::vector<int32_t> ptab;
    int PV = 0, PO = 0, ndblk = 0, nablk = 0;
    int32_t *dptab = nullptr;
    Gemm gp[2];  // packed W_mnij product; both ladders as one packed product
    // packed split operands, rows PV + PO elements long:
    //   pk_A [K][canonical (ki,i,j)]: tau over canonical (ke,e,f) | W_mnij over canonical (km,m,n)
    //   pk_B [K][canonical (ka,a,b)]: dressed <ab||ef> over (ke,e,f) | tau over (km,m,n)
    uint16_t *pk_A = nullptr, *pk_B = nullptr, *pk_oovv = nullptr;
    cd *Lp = nullptr;  // [K][canonical (ki,i,j)][canonical (ka,a,b)]: both ladders' contribution to R2
    double *npart = nullptr;  // per-workgroup sums of |r2|^2 written by the R2 assembly
    // the DIIS extrapolation of the mixed path also leaves the split copy of the new t2 and
    // the energy partial sums at the new amplitudes; these flags say they match the
    // current amplitudes (cleared by every other write of the amplitudes or the inputs)
    double *epart = nullptr;
    bool sp_ok = false, e_ok = false;
    ck::SplitOps sg[5];
    // arithmetic form of each mixed product slot of sg (ck::Arith; slot 2 unused).  The
    // ladder family (slots 0, 1) and the ring family (3, 4) each keep their operands in one
    // storage: split storage while every product of the family is PRESPLIT2, complex64
    // otherwise (a PRESPLIT2 product of a complex64 family then runs as SPLIT2)
    int arith[5] = {ck::ARITH_PRESPLIT2, ck::ARITH_PRESPLIT2, ck::ARITH_PRESPLIT2, ck::ARITH_PRESPLIT2,
                    ck::ARITH_PRESPLIT2};
    // tile shape of each FP64 product (ck::F64Tile, indexed like g)
    int tile[5] = {ck::F64_TILE_64x64, ck::F64_TILE_64x64, ck::F64_TILE_64x64, ck::F64_TILE_64x64,
                   ck::F64_TILE_64x64};
    bool c64_lad() const { return ck::arith_c64(arith[0]) || ck::arith_c64(arith[1]); }
    bool c64_ring() const { return ck::arith_c64(arith[3]) || ck::arith_c64(arith[4]); }
    bool c64_of(int slot) const { return slot < 3 ? c64_lad() : c64_ring(); }
    // k extent of one FP32-accumulated chunk of every mixed product (0: the whole k range;
    // a multiple of 16 otherwise), see run_split_product
    int kchunk = 0;
    // device DIIS state (ck::DiisDev): FIFO head and count, overlaps, new overlaps, coefficients
    int32_t *dstate = nullptr;
    double *dB = nullptr, *dbnew = nullptr, *dcoef = nullptr;
    ck::DiisDev diis() const { return ck::DiisDev{dstate, dB, dbnew, dcoef, desc.diis_space}; }
    bool diis_reset = true;  // the device DIIS state must be cleared before the next update
    // host state
    double rnorm = -1.0;
    bool converged = false, inputs = false;
    // stagnation watch of the mixed path (see watch_stagnation): norm at the last halving
    // and iterations since
    double rn_ref = INFINITY;
    int stall = 0;

    int64_t n1() const { return d.t1(); }
    int64_t n2() const { return d.t2(); }
    cd *t1() const { return amp; }
    cd *t2() const { return amp + n1(); }
    cd *r1() const { return res; }
    cd *r2() const { return mixed ? nullptr : res + n1(); }  // mixed path: r2c
    ck::SysDev dev() const {
        ck::SysDev s;
        s.d = d;
        s.kc = dkc;
        s.eo = eo;
        s.ev = ev;
        s.fock = fock;
        s.oooo = eri[0];
        s.ooov = eri[1];
        s.oovv = eri[2];
        s.ovvo = eri[3];
        s.ovvv = eri[4];
        s.vvvv = eri[5];
        s.ovvoT = ovvoT;
        s.ovvvT = ovvvT;
        s.oovvT = oovvT;
        s.ovvv_c = ovvv_c;
        s.ovvvT_c = ovvvT_c;
        s.ovvoT_c = ovvoT_c;
        s.oovvT_c = oovvT_c;
        s.oovv_c = oovv_c;
        s.oooo_c = oooo_c;
        s.ooov_c = ooov_c;
        s.vvvv_c = vvvv_c;
        s.vblk = mixed ? dblk_dev() + ndblk + nablk : nullptr;
        return s;
    }
    ck::StaticCopies statics() const { return ck::StaticCopies{ovvoT, ovvvT, oovvT}; }
    // offset of dblk in ptab (host) and dptab (device)
    int64_t dblk_off() const {
        const int64_t N = d.N, nv = d.nv, no = d.no;
        return N * (PV + PO) + N * N * (nv * nv + no * no);
    }
    const int32_t *dblk_dev() const { return dptab + dblk_off(); }
    ck::PairTabs pairs() const {
        const int64_t N = d.N;
        const int64_t nv = d.nv;
        const int64_t no = d.no;
        const int32_t *vpos = dptab + N * (PV + PO), *opos = vpos + N * N * nv * nv;
        const int32_t *dblk = opos + N * N * no * no;  // == dblk_dev()
        return ck::PairTabs{dptab, dptab + N * PV, vpos, opos, dblk, dblk + ndblk, PV, PO, ndblk, nablk};
    }
};

struct EventPair {
    hipEvent_t a, b;
    int stage;
};

}  // namespace

struct ccsd_k_ctx {
    std::vector<System> sys;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    uint64_t ws_bytes = 0;
    bool bound = false, failed = false;
    std::string err;
    bool timing = false;
    std::vector<EventPair> pending, pool;
    double stage_ms[ST_COUNT] = {};
    int64_t stage_n[ST_COUNT] = {};
    // streams (default priority, created on first use) on which the systems of a batch run
    // side by side, with the events that order them after and before work on `stream`
    std::vector<hipStream_t> lanes;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> joins;
    bool escalate = true;  // raise stagnating mixed systems to three-term split products
    // iterations replayed from one captured graph (off while stage timing is on); the graph
    // is captured again whenever what it depends on changes (iteration_signature)
    bool graphs = true;
    hipGraphExec_t gexec = nullptr;
    std::vector<int64_t> gsig;
    double *dnorms = nullptr;  // device: ||R||^2 of every system after an iteration
    // A one-system mixed residual runs the side kernels that do not feed the next grouped
    // product (the F sums, the dressed <ab||ef>, the X seed, R1) on a second stream beside
    // the products (default priority, created before any capture); off while stage timing
    // is on, so that every product is timed alone.
    bool overlap = true;
    hipStream_t side = nullptr;
    hipEvent_t sev[4] = {};  // fork, dressed <ab||ef> ready, X seed ready, R1 ready
};

namespace {

int fail(ccsd_k_ctx *c, int code, const std::string &msg) {
    if (c) {
        c->err = msg;
        if (code == CCSD_K_EDEVICE) c->failed = true;
    } else {
        g_init_error = msg;
    }
    return code;
}

int kcons(const ck::Mesh &m, int kp, int kq, int kr) {
    int p2 = kp % m.g2, q2 = kq % m.g2, r2 = kr % m.g2;
    int p1 = (kp / m.g2) % m.g1, q1 = (kq / m.g2) % m.g1, r1 = (kr / m.g2) % m.g1;
    int p0 = kp / (m.g2 * m.g1), q0 = kq / (m.g2 * m.g1), r0 = kr / (m.g2 * m.g1);
    int s0 = ((p0 + q0 - r0) % m.g0 + m.g0) % m.g0;
    int s1 = ((p1 + q1 - r1) % m.g1 + m.g1) % m.g1;
    int s2 = ((p2 + q2 - r2) % m.g2 + m.g2) % m.g2;
    return (s0 * m.g1 + s1) * m.g2 + s2;
}

// ---------------------------------------------------------------- contraction tables
// Canonical pairs of a group of total pair momentum K: (kx, x; ky, y), ky = K - kx, with
// (kx, x) < (ky, y), listed by kx, x, y; every group padded to the same length (a multiple
// of 16) so that the grouped products have one k extent.  Packed ladder products (mixed
// path), on canonical pairs in rows, columns and k alike (antisymmetry, pack.hip): an
// eighth of the full form's work each.
//   G1p: W_mnij += tau . <mn||ef>^T   rows canonical (ki,i,j), cols canonical (km,m,n),
//        k canonical (ke,e,f) (alpha 1 = 1/2 x 2 for the canonical k pairs); written split
//        into the W_mnij part of pk_A
//   G23p: L = tau . Vt^T + W_mnij . tauT   rows canonical (ki,i,j), cols canonical (ka,a,b),
//        k = canonical (ke,e,f) then canonical (km,m,n): both ladders as one product on
//        the concatenated rows of pk_A and pk_B, written (beta 0) to the packed Lp; the
//        assembly of R2 expands it to all four orientations of the two pairs.
void build_tables(System &S);
void build_pair_tables(System &S) {
    const int64_t N = S.d.N, o = S.d.no, v = S.d.nv;
    const int64_t oo = o * o, vv = v * v, o4 = oo * oo;
    auto kc = [&](int64_t a, int64_t b, int64_t c) { return (int64_t)S.kc[(a * N + b) * N + c]; };
    auto list = [&](int64_t K, int64_t w, std::vector<int32_t> &out) {
        out.clear();
        for (int64_t kx = 0; kx < N; ++kx) {
            const int64_t ky = kc(K, 0, kx);
            if (kx > ky) continue;
            for (int64_t x = 0; x < w; ++x)
                for (int64_t y = (kx == ky ? x + 1 : 0); y < w; ++y) out.push_back((int32_t)((kx * w + x) * w + y));
        }
    };
    std::vector<std::vector<int32_t>> vl(N), ol(N);
    size_t mv = 0, mo = 0;
    for (int64_t K = 0; K < N; ++K) {
        list(K, v, vl[K]);
        list(K, o, ol[K]);
        mv = std::max(mv, vl[K].size());
        mo = std::max(mo, ol[K].size());
    }
    S.PV = (int)((mv + 15) / 16 * 16);
    S.PO = (int)((mo + 15) / 16 * 16);
    if (S.PV == 0) S.PV = 16;
    if (S.PO == 0) S.PO = 16;
    const int64_t PV = S.PV, PO = S.PO;
    std::vector<int32_t> dblk;
    for (int64_t ka = 0; ka < N; ++ka)
        for (int64_t kb = ka; kb < N; ++kb)
            for (int64_t ke = 0; ke < N; ++ke)
                if (ke <= kc(ka, kb, ke)) dblk.push_back((int32_t)((ka * N + kb) * N + ke));
    S.ndblk = (int)dblk.size();
    // R2 blocks (ki, kj, ka) that represent their orbit under (ki <-> kj) and (ka <-> kb):
    // ki <= kj and ka <= kb (the assembly writes the other members)
    std::vector<int32_t> ablk;
    for (int64_t ki = 0; ki < N; ++ki)
        for (int64_t kj = ki; kj < N; ++kj)
            for (int64_t ka = 0; ka < N; ++ka)
                if (ka <= kc(ki, kj, ka)) ablk.push_back((int32_t)((ki * N + kj) * N + ka));
    S.nablk = (int)ablk.size();
    S.ptab.assign(N * PV + N * PO + N * N * vv + N * N * oo, -1);
    S.ptab.insert(S.ptab.end(), dblk.begin(), dblk.end());
    S.ptab.insert(S.ptab.end(), ablk.begin(), ablk.end());
    std::vector<int32_t> vblk(N * N * N, -1);
    for (size_t L = 0; L < dblk.size(); ++L) vblk[dblk[L]] = (int32_t)L;
    S.ptab.insert(S.ptab.end(), vblk.begin(), vblk.end());
    int32_t *vlist = S.ptab.data(), *olist = vlist + N * PV, *vpos = olist + N * PO, *opos = vpos + N * N * vv;
    for (int64_t K = 0; K < N; ++K) {
        for (size_t p = 0; p < vl[K].size(); ++p) {
            vlist[K * PV + p] = vl[K][p];
            const int64_t kx = vl[K][p] / vv, xy = vl[K][p] % vv;
            vpos[(K * N + kx) * vv + xy] = (int32_t)p;
        }
        for (size_t p = 0; p < ol[K].size(); ++p) {
            olist[K * PO + p] = ol[K][p];
            const int64_t kx = ol[K][p] / oo, xy = ol[K][p] % oo;
            opos[(K * N + kx) * oo + xy] = (int32_t)p;
        }
    }
    std::vector<int64_t> &T = S.tables;
    auto put = [&](Gemm &g, int which, int64_t len, auto fn) {
        g.tab[which] = T.size();
        for (int64_t x = 0; x < len; ++x) T.push_back(fn(x));
    };
    Gemm &g1 = S.gp[0], &g2 = S.gp[1];
    const int64_t R = PV + PO;  // row length of pk_A and pk_B
    // W_mnij row of canonical (ki,i,j) = pr of group K, -1 for the padding (no output)
    auto row_wt = [&](int64_t K, int32_t pr) {
        if (pr < 0) return (int64_t)-1;
        int64_t ki = pr / oo, ij = pr % oo;
        return ((ki * N + kc(K, 0, ki)) * N) * o4 + ij * oo;
    };
    // G1p
    put(g1, 0, N * PO, [&](int64_t x) { return x * R; });  // tau part of pk_A
    put(g1, 1, N * PV, [&](int64_t x) { return x % PV; });
    put(g1, 2, N * PO, [&](int64_t x) { return x * PV; });  // oovv_pk rows
    g1.tab[3] = g1.tab[1];
    put(g1, 4, N * PO, [&](int64_t x) { return row_wt(x / PO, olist[x]); });
    put(g1, 5, N * PO, [&](int64_t x) {  // W_mnij column of canonical (km,m,n), -1 in the padding
        const int32_t pr = olist[x];
        if (pr < 0) return (int64_t)-1;
        return (int64_t)(pr / oo) * o4 + pr % oo;
    });
    g1.cs_row = T.size();  // W_mnij part of pk_A
    for (int64_t x = 0; x < N * PO; ++x) T.push_back(x * R + PV);
    g1.cs_col = T.size();
    for (int64_t x = 0; x < N * PO; ++x) T.push_back(x % PO);
    g1.op.G = (int)N; g1.op.M = (int)PO; g1.op.N = (int)PO; g1.op.K = (int)PV;
    g1.op.alpha = 1.0; g1.op.beta = 1.0; g1.stage = ST_WMN;
    // G23p
    g2.tab[0] = g1.tab[0];
    put(g2, 1, N * R, [&](int64_t x) { return x % R; });
    put(g2, 2, N * PV, [&](int64_t x) { return x * R; });  // pk_B rows
    g2.tab[3] = g2.tab[1];
    put(g2, 4, N * PO, [&](int64_t x) { return olist[x] < 0 ? (int64_t)-1 : x * PV; });  // Lp rows
    put(g2, 5, N * PV, [&](int64_t x) { return vlist[x] < 0 ? (int64_t)-1 : x % PV; });
    g2.op.G = (int)N; g2.op.M = (int)PO; g2.op.N = (int)PV; g2.op.K = (int)R;
    g2.op.alpha = 1.0; g2.op.beta = 0.0; g2.stage = ST_PP;
}

// Offsets in complex elements.  Group label: total pair momentum K for the ladder
// family, momentum transfer q for the ring family.
void build_tables(System &S) {
    const int64_t N = S.d.N, o = S.d.no, v = S.d.nv;
    const int64_t oo = o * o, vv = v * v, ov = o * v, t2b = oo * vv, o4 = oo * oo, v4 = vv * vv;
    auto kc = [&](int a, int b, int c) { return (int64_t)S.kc[((int64_t)a * N + b) * N + c]; };
    std::vector<int64_t> &T = S.tables;
    T.clear();
    auto put = [&](Gemm &g, int which, int64_t len, auto fn) {
        g.tab[which] = T.size();
        for (int64_t x = 0; x < len; ++x) T.push_back(fn(x));
    };
    const int64_t Mpp = N * oo, Npp = N * vv, Mph = N * ov;

    // G1: W_mnij(T) += 1/2 tau . <mn||ef>^T       rows (ki,i,j), cols (km,m,n), k (ke,e,f)
    // G2: r2 += 1/2 tau . Vt^T                      rows (ki,i,j), cols (ka,a,b), k (ke,e,f)
    // G3: r2 += 1/2 W_mnij(T) . tauT                rows (ki,i,j), cols (ka,a,b), k (km,m,n)
    auto row_t2 = [&](int64_t K, int64_t x) {  // (ki,i,j) -> t2/r2 block [ki][K-ki][.]
        int64_t ki = x / oo, ij = x % oo;
        return ((ki * N + kc(K, 0, ki)) * N) * t2b + ij * vv;
    };
    auto row_wt = [&](int64_t K, int64_t x) {
        int64_t ki = x / oo, ij = x % oo;
        return ((ki * N + kc(K, 0, ki)) * N) * o4 + ij * oo;
    };
    Gemm &g1 = S.g[0], &g2 = S.g[1], &g3 = S.g[2], &g4 = S.g[3], &g5 = S.g[4];
    put(g1, 0, N * Mpp, [&](int64_t x) { return row_t2(x / Mpp, x % Mpp); });
    put(g1, 1, N * Npp, [&](int64_t x) { int64_t y = x % Npp; return (y / vv) * t2b + y % vv; });
    put(g1, 2, N * Mpp, [&](int64_t x) {
        int64_t K = x / Mpp, y = x % Mpp, km = y / oo;
        return ((km * N + kc(K, 0, km)) * N) * t2b + (y % oo) * vv;
    });
    g1.tab[3] = g1.tab[1];
    put(g1, 4, N * Mpp, [&](int64_t x) { return row_wt(x / Mpp, x % Mpp); });
    put(g1, 5, N * Mpp, [&](int64_t x) { int64_t y = x % Mpp; return (y / oo) * o4 + y % oo; });
    g1.op.G = (int)N; g1.op.M = (int)Mpp; g1.op.N = (int)Mpp; g1.op.K = (int)Npp;
    g1.op.alpha = 0.5; g1.op.beta = 1.0; g1.stage = ST_WMN;

    g2.tab[0] = g1.tab[0];
    g2.tab[1] = g1.tab[1];
    put(g2, 2, N * Npp, [&](int64_t x) {
        int64_t K = x / Npp, y = x % Npp, ka = y / vv;
        return ((ka * N + kc(K, 0, ka)) * N) * v4 + (y % vv) * vv;
    });
    put(g2, 3, N * Npp, [&](int64_t x) { int64_t y = x % Npp; return (y / vv) * v4 + y % vv; });
    g2.tab[4] = g1.tab[0];
    put(g2, 5, N * Npp, [&](int64_t x) { int64_t y = x % Npp; return (y / vv) * t2b + y % vv; });
    g2.op.G = (int)N; g2.op.M = (int)Mpp; g2.op.N = (int)Npp; g2.op.K = (int)Npp;
    g2.op.alpha = 0.5; g2.op.beta = 1.0; g2.stage = ST_PP;

    g3.tab[0] = g1.tab[4];
    g3.tab[1] = g1.tab[5];
    put(g3, 2, N * Npp, [&](int64_t x) { int64_t y = x % Npp; return (y / vv) * t2b + (y % vv) * oo; });
    put(g3, 3, N * Mpp, [&](int64_t x) {
        int64_t K = x / Mpp, y = x % Mpp, km = y / oo;
        return ((km * N + kc(K, 0, km)) * N) * t2b + y % oo;
    });
    g3.tab[4] = g2.tab[4];
    g3.tab[5] = g2.tab[5];
    g3.op.G = (int)N; g3.op.M = (int)Mpp; g3.op.N = (int)Npp; g3.op.K = (int)Mpp;
    g3.op.alpha = 0.5; g3.op.beta = 1.0; g3.stage = ST_HH;

    // G4: WR += 1/2 t_{jn}^{bf} <mn||ef>   rows (kj,j,b), cols (km,m,e), k (kn,n,f)
    // G5: X  += t_{im}^{ae} W_mbej          rows (ki,i,a), cols (kj,j,b), k (km,m,e)
    put(g4, 0, N * Mph, [&](int64_t x) {
        int64_t q = x / Mph, y = x % Mph, kj = y / ov, j = (y % ov) / v, b = y % v;
        return (kj * N * N + kc(kj, 0, q)) * t2b + j * o * vv + b * v;
    });
    put(g4, 1, N * Mph, [&](int64_t x) {
        int64_t y = x % Mph, kn = y / ov, n = (y % ov) / v, f = y % v;
        return kn * N * t2b + n * vv + f;
    });
    put(g4, 2, N * Mph, [&](int64_t x) {
        int64_t q = x / Mph, y = x % Mph, km = y / ov, m = (y % ov) / v, e = y % v;
        return (km * N * N + kc(km, 0, q)) * t2b + m * o * vv + e * v;
    });
    g4.tab[3] = g4.tab[1];
    put(g4, 4, N * Mph, [&](int64_t x) {
        int64_t q = x / Mph, y = x % Mph, kj = y / ov;
        return ((q * N + kj) * N) * ov * ov + (y % ov) * ov;
    });
    put(g4, 5, N * Mph, [&](int64_t x) { int64_t y = x % Mph; return (y / ov) * ov * ov + y % ov; });
    g4.op.G = (int)N; g4.op.M = (int)Mph; g4.op.N = (int)Mph; g4.op.K = (int)Mph;
    g4.op.alpha = 0.5; g4.op.beta = 1.0; g4.stage = ST_WR;

    put(g5, 0, N * Mph, [&](int64_t x) {
        int64_t q = x / Mph, y = x % Mph, ki = y / ov, i = (y % ov) / v, a = y % v;
        return (ki * N * N + kc(ki, q, 0)) * t2b + i * o * vv + a * v;
    });
    put(g5, 1, N * Mph, [&](int64_t x) {
        int64_t y = x % Mph, km = y / ov, m = (y % ov) / v, e = y % v;
        return km * N * t2b + m * vv + e;
    });
    g5.tab[2] = g4.tab[4];
    g5.tab[3] = g4.tab[5];
    put(g5, 4, N * Mph, [&](int64_t x) {
        int64_t q = x / Mph, y = x % Mph, ki = y / ov;
        return ((q * N + ki) * N) * ov * ov + (y % ov) * ov;
    });
    put(g5, 5, N * Mph, [&](int64_t x) { int64_t y = x % Mph; return (y / ov) * ov * ov + y % ov; });
    g5.op.G = (int)N; g5.op.M = (int)Mph; g5.op.N = (int)Mph; g5.op.K = (int)Mph;
    g5.op.alpha = 1.0; g5.op.beta = 1.0; g5.stage = ST_RING;
    // the pair tables serve the packed products of the mixed path and the packed DIIS
    // history of both paths
    build_pair_tables(S);
}

// ---------------------------------------------------------------- workspace plan
struct Carver {
    uintptr_t base, off = 0;
    bool assign;
    template <class T>
    void take(T *&p, int64_t count) {
        off = (off + 255) & ~(uintptr_t)255;
        if (assign) p = reinterpret_cast<T *>(base + off);
        off += (uintptr_t)count * sizeof(T);
    }
};

void carve(System &S, Carver &c) {
    const int64_t N = S.d.N, o = S.d.no, v = S.d.nv, n = o + v, N3 = N * N * N;
    const int64_t cls[6] = {o * o * o * o, o * o * o * v, o * o * v * v, o * v * v * o, o * v * v * v, v * v * v * v};
    c.take(S.fock, N * n * n);
    if (!S.mixed)
        for (int i = 0; i < 6; ++i) c.take(S.eri[i], N3 * cls[i]);
    c.take(S.amp, S.n1() + S.n2());
    c.take(S.res, S.mixed ? S.n1() : S.n1() + S.n2());
    if (S.mixed) c.take(S.r2c, S.n2());
    if (!S.mixed) {
        c.take(S.tau, S.n2());
        c.take(S.tauT, S.n2());
        c.take(S.Vt, N3 * cls[5]);
    } else {
        // split storage: 4 bf16 per element
        S.pl_t2 = (S.n2() + 63) / 64 * 64;
        const int64_t PV = S.PV, PO = S.PO;
        c.take(S.sp_t2, 4 * S.pl_t2);
        c.take(S.sp_WR, 4 * S.pl_t2);
        c.take(S.sp_oovv, 4 * S.pl_t2);
        c.take(S.pk_A, 4 * N * PO * (PV + PO));
        c.take(S.pk_B, 4 * N * PV * (PV + PO));
        c.take(S.pk_oovv, 4 * N * PO * PV);
        c.take(S.Lp, N * PO * PV);
        c.take(S.npart, ck::assemble_pack_blocks(S.d, S.pairs()));
        c.take(S.epart, 2 + 2 * ck::lincomb_pack_blocks(S.d, S.pairs()));
    }
    c.take(S.dptab, (int64_t)S.ptab.size());
    c.take(S.WT, N3 * cls[0]);
    if (S.rearranged()) {
        c.take(S.t2T, S.n2());
        c.take(S.XT, N3 * cls[0]);
    }
    c.take(S.WR, N3 * o * v * o * v);
    c.take(S.X, N3 * o * v * o * v);
    c.take(S.scr, N3 * o * o * o * v);
    if (S.mixed) c.take(S.scrq, N3 * o * o * o * v);  // the X seed's Q beside the W seed's Z
    if (S.mixed) {
        c.take(S.ovvoT_c, S.n2());
        c.take(S.ovvv_c, N3 * cls[4]);
        c.take(S.ovvvT_c, N3 * cls[4]);
        c.take(S.oovv_c, S.n2());
        c.take(S.oovvT_c, S.n2());
        c.take(S.oooo_c, N3 * cls[0]);
        c.take(S.ooov_c, N3 * cls[1]);
        c.take(S.vvvv_c, (int64_t)S.ndblk * cls[5]);
    } else {
        c.take(S.ovvoT, S.n2());
        c.take(S.ovvvT, N3 * cls[4]);
        c.take(S.oovvT, S.n2());
    }
    const int64_t fs = ck::fr_splits(S.d);  // slices of the F and R1 block-sum partials
    c.take(S.P1, 2 * fs * N3 * o * v);
    c.take(S.fw.Fov, N * o * v);
    c.take(S.fw.Foo, N * o * o);
    c.take(S.fw.Fvv, N * v * v);
    c.take(S.fw.Fot, N * o * o);
    c.take(S.fw.Fvt, N * v * v);
    c.take(S.fw.Poo, fs * N3 * o * o);
    c.take(S.fw.Pvv, fs * N3 * v * v);
    c.take(S.zeros, 16);
    c.take(S.eo, N * o);
    c.take(S.ev, N * v);
    c.take(S.red, 16 * (int64_t)ck::UPD_BLOCKS);
    c.take(S.redout, 32);
    c.take(S.dkc, N3);
    c.take(S.dtab, (int64_t)S.tables.size());
    const int md = std::max(S.desc.diis_space, 1);
    c.take(S.dstate, 4);
    c.take(S.dB, md * md);
    c.take(S.dbnew, md);
    c.take(S.dcoef, md);
    // the DIIS history pointers are written only when assigning: a size query (assign
    // false) on a bound context must leave them intact
    const int m = S.desc.diis_space;
    if (c.assign) {
        S.dvec.assign(m, nullptr);
        S.derr.assign(S.mixed ? 0 : m, nullptr);
        S.derr32.assign(S.mixed ? m : 0, nullptr);
    }
    // packed history (t1 in full, t2 on the antisymmetry-orbit representatives); error
    // vectors in complex64 on the mixed path, complex128 on the FP64 path
    const int64_t hl = ck::packed_len(S.d, S.pairs());
    for (int i = 0; i < m; ++i) {
        cd *vec = nullptr, *err = nullptr;
        ck::cf *err32 = nullptr;
        c.take(vec, hl);
        if (S.mixed) c.take(err32, hl);
        else c.take(err, hl);
        if (!c.assign) continue;
        S.dvec[i] = vec;
        if (S.mixed) S.derr32[i] = err32;
        else S.derr[i] = err;
    }
}

// True when every aligned group of 8 k indices of both operands is a contiguous,
// 16-byte aligned run in every group, and all row/column bases are 8-aligned.
bool fast_ok(const System &S, const Gemm &g) {
    const int64_t G = g.op.G, M = g.op.M, N = g.op.N, K = g.op.K;
    if (K % 8) return false;
    const int64_t *T = S.tables.data();
    for (int64_t x = 0; x < G * M; ++x)
        if (T[g.tab[0] + x] % 8) return false;
    for (int64_t x = 0; x < G * N; ++x)
        if (T[g.tab[2] + x] % 8) return false;
    for (int w : {1, 3})
        for (int64_t gg = 0; gg < G; ++gg)
            for (int64_t k0 = 0; k0 < K; k0 += 8) {
                const int64_t *r = T + g.tab[w] + gg * K + k0;
                if (r[0] % 8) return false;
                for (int j = 1; j < 8; ++j)
                    if (r[j] != r[0] + j) return false;
            }
    return true;
}

void bind_ops(System &S) {
    const int64_t *T = S.dtab;
    const cd *A[5] = {S.tau, S.tau, S.WT, S.t2(), S.t2()};
    const cd *Bm[5] = {S.eri[2], S.Vt, S.tauT, S.eri[2], S.WR};
    cd *C[5] = {S.WT, S.r2(), S.r2(), S.WR, S.X};
    for (int i = 0; i < 5; ++i) {
        Gemm &g = S.g[i];
        g.op.A = A[i];
        g.op.B = Bm[i];
        g.op.C = C[i];
        g.op.a_row = T + g.tab[0];
        g.op.a_k = T + g.tab[1];
        g.op.b_col = T + g.tab[2];
        g.op.b_k = T + g.tab[3];
        g.op.c_row = T + g.tab[4];
        g.op.c_col = T + g.tab[5];
        g.op.zeros = S.zeros;
    }
    if (S.rearranged()) {
        // X-tilde = t2 . <mn||ef>^T (the W_mnij product on t2, alpha 1, into XT); the two
        // hole-hole products on the transposed t2: r2 += 1/4 X-tilde t2T and r2 += Y t2T
        S.gr[0] = S.g[0];
        S.gr[0].op.A = S.t2();
        S.gr[0].op.C = S.XT;
        S.gr[0].op.alpha = 1.0;
        S.gr[0].op.beta = 0.0;
        S.gr[1] = S.g[2];
        S.gr[1].op.A = S.XT;
        S.gr[1].op.B = S.t2T;
        S.gr[1].op.alpha = 0.25;
        S.gr[2] = S.g[2];
        S.gr[2].op.A = S.WT;
        S.gr[2].op.B = S.t2T;
        S.gr[2].op.alpha = 1.0;
    }
    if (!S.mixed) return;
    // the ladder family on packed pairs (gp: W_mnij, then both ladders as one product; slot
    // 2, the separate hole-hole product, is unused), the ring family in full (g[3], g[4])
    const Gemm *G[5] = {&S.gp[0], &S.gp[1], &S.gp[1], &S.g[3], &S.g[4]};
    const uint16_t *SA[5] = {S.pk_A, S.pk_A, S.pk_A, S.sp_t2, S.sp_t2};
    const uint16_t *SB[5] = {S.pk_oovv, S.pk_B, S.pk_B, S.sp_oovv, S.sp_WR};
    // W_mnij and W_mbej are only consumed as split operands: their products write split
    uint16_t *CS[5] = {S.pk_A, nullptr, nullptr, S.sp_WR, nullptr};
    auto tab = [&](size_t off) { return off == SIZE_MAX ? nullptr : T + off; };
    for (int i = 0; i < 5; ++i) {
        const Gemm &g = *G[i];
        ck::SplitOps &s = S.sg[i];
        s = ck::SplitOps{};
        s.A = SA[i];
        s.B = SB[i];
        s.zeros = reinterpret_cast<const uint16_t *>(S.zeros);
        s.C = i == 1 || i == 2 ? S.Lp : C[i];  // the ladders write the packed Lp
        s.Cs = CS[i];
        s.a_row = T + g.tab[0]; s.a_k = T + g.tab[1]; s.b_col = T + g.tab[2]; s.b_k = T + g.tab[3];
        s.c_row = T + g.tab[4]; s.c_col = T + g.tab[5];
        s.cs_row = tab(g.cs_row); s.cs_col = tab(g.cs_col);
        s.G = g.op.G; s.M = g.op.M; s.N = g.op.N; s.K = g.op.K; s.alpha = g.op.alpha; s.beta = g.op.beta;
        s.fast = fast_ok(S, g) ? 1 : 0;
    }
}

// ---------------------------------------------------------------- timing
void stage_begin(ccsd_k_ctx *c, EventPair &ep, int stage, hipStream_t st = nullptr) {
    if (!c->timing) return;
    if (!st) st = c->stream;
    if (c->pool.empty()) {
        EventPair p;
        CK_CHECK(hipEventCreate(&p.a));
        CK_CHECK(hipEventCreate(&p.b));
        c->pool.push_back(p);
    }
    ep = c->pool.back();
    c->pool.pop_back();
    ep.stage = stage;
    CK_CHECK(hipEventRecord(ep.a, st));
}
void stage_end(ccsd_k_ctx *c, EventPair &ep, hipStream_t st = nullptr) {
    if (!c->timing) return;
    CK_CHECK(hipEventRecord(ep.b, st ? st : c->stream));
    c->pending.push_back(ep);
}
void collect_timing(ccsd_k_ctx *c) {
    if (c->pending.empty()) return;
    CK_CHECK(hipStreamSynchronize(c->stream));
    for (auto &p : c->pending) {
        float ms = 0.f;
        CK_CHECK(hipEventElapsedTime(&ms, p.a, p.b));
        c->stage_ms[p.stage] += ms;
        c->stage_n[p.stage] += 1;
        c->pool.push_back(p);
    }
    c->pending.clear();
}

// ---------------------------------------------------------------- systems side by side
// (eight streams: the 96-system batch measured 183 ms per iteration against 192 with four;
// twelve and sixteen measured the same as eight)
constexpr int NLANES = 8;

// The streams for a set of systems: the context's own stream for one system; for several,
// the lanes, each system to the lane with the least work so far (largest first, work
// taken as N^4 (o v)^2 (o + v)^2 plus a fixed per-system part for its ~40 launches), after
// a fork event on the context's stream.  join_lanes orders the context's stream after them.
std::vector<hipStream_t> fork_lanes(ccsd_k_ctx *c, const std::vector<System *> &sys) {
    std::vector<hipStream_t> out(sys.size(), c->stream);
    if (sys.size() < 2) return out;
    if (c->lanes.empty()) {  // all or nothing: a failed creation leaves no partial set
        hipEvent_t fork = nullptr;
        std::vector<hipStream_t> lanes(NLANES, nullptr);
        std::vector<hipEvent_t> joins(NLANES, nullptr);
        hipError_t err = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
        for (int l = 0; err == hipSuccess && l < NLANES; ++l) {
            err = hipStreamCreateWithFlags(&lanes[l], hipStreamNonBlocking);
            if (err == hipSuccess) err = hipEventCreateWithFlags(&joins[l], hipEventDisableTiming);
        }
        if (err != hipSuccess) {
            for (hipStream_t st : lanes)
                if (st) (void)hipStreamDestroy(st);
            for (hipEvent_t ev : joins)
                if (ev) (void)hipEventDestroy(ev);
            if (fork) (void)hipEventDestroy(fork);
            throw ck::HipError(err, "creating the streams of systems side by side", __FILE__, __LINE__);
        }
        c->fork = fork;
        c->lanes = lanes;
        c->joins = joins;
    }
    CK_CHECK(hipEventRecord(c->fork, c->stream));
    for (hipStream_t st : c->lanes) CK_CHECK(hipStreamWaitEvent(st, c->fork, 0));
    std::vector<double> work(sys.size());
    std::vector<size_t> order(sys.size());
    for (size_t k = 0; k < sys.size(); ++k) {
        const double N = sys[k]->d.N, o = sys[k]->d.no, v = sys[k]->d.nv;
        work[k] = N * N * N * N * (o * v) * (o * v) * (o + v) * (o + v) + 2e8;
        order[k] = k;
    }
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return work[a] > work[b]; });
    double load[NLANES] = {};
    for (size_t k : order) {
        const int l = (int)(std::min_element(load, load + NLANES) - load);
        load[l] += work[k];
        out[k] = c->lanes[l];
    }
    return out;
}
void join_lanes(ccsd_k_ctx *c, const std::vector<hipStream_t> &used) {
    if (used.size() < 2) return;
    for (int l = 0; l < NLANES; ++l) {
        CK_CHECK(hipEventRecord(c->joins[l], c->lanes[l]));
        CK_CHECK(hipStreamWaitEvent(c->stream, c->joins[l], 0));
    }
}

void apply_form(ccsd_k_ctx *c, System &S, int slot, int a);

// Precision escalation of the mixed path.  The products carry rounding errors that change
// from one iteration to the next (the two-term split ~2^-16 relative per product, FP32
// accumulation ~2^-24 sqrt(steps) of the running sum), so the residual of a mixed system
// has a floor that grows with the coupling strength; a system whose residual norm has not
// halved for three iterations while still above the tolerance is at that floor.  Every
// product it runs in a two-term form is then raised to the three-term split, and every
// product accumulates in FP32 over chunks of 256 k only, adding the chunks in FP64; a
// second stall shortens the chunks to 64 k.
void watch_stagnation(ccsd_k_ctx *c, System &S) {
    if (!S.mixed) return;
    if (S.rnorm < 0.5 * S.rn_ref) {
        S.rn_ref = S.rnorm;
        S.stall = 0;
        return;
    }
    if (++S.stall < 3) return;
    S.stall = 0;
    S.rn_ref = S.rnorm;
    if (S.kchunk == 0) {
        for (int slot : {0, 1, 3, 4})
            if (S.arith[slot] == ck::ARITH_PRESPLIT2 || S.arith[slot] == ck::ARITH_SPLIT2)
                apply_form(c, S, slot, ck::ARITH_SPLIT3);
        S.kchunk = 256;
    } else if (S.kchunk > 64) {
        S.kchunk = 64;  // a second stall: chunks of 64 k
    }
}

// product slot i of the mixed path in its arithmetic form, on its family's storage.  With
// S.kchunk > 0 the k range is summed in chunks of that many k: FP32 accumulation spans one
// chunk and the chunks are added in FP64.  On complex64 storage (every product of an
// escalated system) that is one launch that keeps the FP64 sums in registers; on split
// storage each chunk is a launch that adds its part to the FP64 output (the first with the
// product's beta, the rest with 1; only the last writes the split copy).
void run_split_product(System &S, int i, hipStream_t st) {
    const bool c64 = S.c64_of(i);
    const int a = !c64 ? (int)ck::ARITH_PRESPLIT2
                       : (S.arith[i] == ck::ARITH_PRESPLIT2 ? (int)ck::ARITH_SPLIT2 : S.arith[i]);
    auto launch = [&](const ck::SplitOps &o) {
        if (c64) ck::gemm_c64(o, a, st);
        else ck::gemm_split(o, st);
    };
    const ck::SplitOps &op = S.sg[i];
    const int kc = S.kchunk;
    if (kc <= 0 || op.K <= kc) {
        launch(op);
        return;
    }
    if (c64) {
        ck::gemm_c64_chunked(op, a, kc, st);
        return;
    }
    for (int k0 = 0; k0 < op.K; k0 += kc) {
        ck::SplitOps o = op;
        o.kld = op.K;
        o.a_k = op.a_k + k0;
        o.b_k = op.b_k + k0;
        o.K = std::min(kc, op.K - k0);
        o.beta = k0 == 0 ? op.beta : 1.0;
        if (k0 + kc < op.K) o.Cs = nullptr;
        launch(o);
    }
}

void run_op(ccsd_k_ctx *c, const Gemm &g, int stage, hipStream_t st) {
    EventPair ep{};
    stage_begin(c, ep, stage, st);
    ck::gemm_f64(g.op, st);
    stage_end(c, ep, st);
}

void run_gemm(ccsd_k_ctx *c, System &S, int i, hipStream_t st) {
    EventPair ep{};
    stage_begin(c, ep, (S.mixed && i < 2 ? S.gp[i] : S.g[i]).stage, st);
    if (S.mixed) run_split_product(S, i, st);
    else ck::gemm_f64_tile(S.g[i].op, S.tile[i], st);
    stage_end(c, ep, st);
}

// The second stream of a one-system mixed residual and its events, created once, outside
// any capture (all or nothing).
void ensure_side(ccsd_k_ctx *c) {
    if (c->side || !c->overlap) return;
    bool any = false;
    for (const System &S : c->sys) any = any || S.mixed;
    if (!any) return;
    hipStream_t st = nullptr;
    hipEvent_t ev[4] = {};
    hipError_t err = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    for (int i = 0; err == hipSuccess && i < 4; ++i) err = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming);
    if (err != hipSuccess) {
        if (st) (void)hipStreamDestroy(st);
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
        throw ck::HipError(err, "creating the side stream of the mixed residual", __FILE__, __LINE__);
    }
    c->side = st;
    for (int i = 0; i < 4; ++i) c->sev[i] = ev[i];
}

// The side stream for a residual of S on st, or null to run everything on st: only for a
// mixed system on the context's own stream (one active system) with stage timing off.
hipStream_t side_stream(ccsd_k_ctx *c, const System &S, hipStream_t st) {
    if (!S.mixed || !c->overlap || !c->side || c->timing || st != c->stream) return nullptr;
    return c->side;
}

// One evaluation of (R1, R2) at the current amplitudes, left in S.res, on stream st.
void residual_device(ccsd_k_ctx *c, System &S, hipStream_t st) {
    ck::SysDev s = S.dev();
    EventPair all{};
    stage_begin(c, all, ST_RES, st);
    if (!S.mixed && S.rearranged()) {
        // the hole-hole part in the grouping of Sec. 3.3.4: X-tilde = t2 <mn||ef>,
        // 1/4 t2 X-tilde and t2 Y-tilde_{mnij} as separate products, tau's single-amplitude
        // part of the hole-hole ladder by a small kernel; everything else as below
        ck::launch_tau(s, S.t1(), S.t2(), S.tau, nullptr, st);
        ck::launch_block_transpose(S.d, S.t2(), S.t2T, st);
        ck::launch_f(s, S.t1(), S.t2(), S.fw, st);
        ck::launch_wmnij_init(s, S.t1(), S.WT, false, st);
        ck::launch_ytilde(s, S.t1(), S.WT, st);
        run_op(c, S.gr[0], ST_WMN, st);  // X-tilde
        ck::launch_vvvv_dress(s, S.t1(), S.Vt, st);
        ck::launch_ring_init(s, S.t1(), S.t2(), S.fw, S.scr, S.WR, S.X, st);
        run_gemm(c, S, 3, st);
        run_gemm(c, S, 4, st);
        ck::launch_assemble_r2(s, S.X, S.r2(), st);
        run_gemm(c, S, 1, st);  // particle-particle ladder
        run_op(c, S.gr[1], ST_HH, st);  // A-tilde: 1/4 t2 X-tilde
        run_op(c, S.gr[2], ST_HH, st);  // t2 Y-tilde_{mnij}
        ck::launch_hh_t1_rest(s, S.t1(), S.WT, S.XT, S.r2(), st);
        ck::launch_r1(s, S.t1(), S.t2(), S.fw, S.P1, S.r1(), st);
    } else if (!S.mixed) {
        ck::launch_tau(s, S.t1(), S.t2(), S.tau, S.tauT, st);
        ck::launch_f(s, S.t1(), S.t2(), S.fw, st);
        ck::launch_wmnij_init(s, S.t1(), S.WT, false, st);
        run_gemm(c, S, 0, st);  // W_mnij += 1/2 tau <mn||ef>
        ck::launch_vvvv_dress(s, S.t1(), S.Vt, st);
        ck::launch_ring_init(s, S.t1(), S.t2(), S.fw, S.scr, S.WR, S.X, st);
        run_gemm(c, S, 3, st);  // W_mbej += 1/2 t2 <mn||ef>
        run_gemm(c, S, 4, st);  // X += t2 W_mbej
        ck::launch_assemble_r2(s, S.X, S.r2(), st);
        run_gemm(c, S, 1, st);  // particle-particle ladder
        run_gemm(c, S, 2, st);  // hole-hole ladder
        ck::launch_r1(s, S.t1(), S.t2(), S.fw, S.P1, S.r1(), st);
    } else {
        // Two chains after the F sums: the products with their seeds (tau, the W_mnij and
        // W_mbej seeds), and the side kernels (the X seed's Q and one-pass seed, the dressed
        // <ab||ef>, R1), which meet the first at the ring and ladder products and at the end.
        // With a side stream the second chain is forked when the W_mbej product is issued,
        // so that it runs beside that product instead of delaying the seeds before it;
        // without one, everything runs on st in one order. Every kernel writes buffers the other chain neither reads nor writes
        // (the dressing and tau write disjoint 64-byte chunks of pk_B), so the results are
        // the same.
        const int64_t R = S.PV + S.PO;
        const hipStream_t sb = side_stream(c, S, st);
        if (!S.sp_ok) ck::launch_operand(S.n2(), S.t2(), S.sp_t2, S.c64_ring(), st);
        S.sp_ok = true;
        ck::launch_tau_pack(S.d, S.dkc, S.pairs(), S.t1(), S.t2(), S.pk_A, R, S.pk_B + 4 * (int64_t)S.PV, R,
                            S.c64_lad(), st);
        ck::launch_wmnij_init(s, S.t1(), S.WT, true, st);
        run_gemm(c, S, 0, st);  // W_mnij += 1/2 tau <mn||ef>, written split into pk_A
        ck::launch_f(s, S.t1(), S.t2(), S.fw, st);
        ck::launch_ring_w(s, S.t1(), S.scr, S.WR, st);
        auto side = [&](hipStream_t s2) {
            ck::launch_ring_x(s, S.t1(), S.t2(), S.fw, S.scrq, S.X, s2);
            if (sb) CK_CHECK(hipEventRecord(c->sev[2], sb));
            ck::launch_vvvv_dress_pack(s, S.pairs(), S.t1(), S.pk_B, R, S.c64_lad(), s2);
            if (sb) CK_CHECK(hipEventRecord(c->sev[1], sb));
            ck::launch_r1(s, S.t1(), S.t2(), S.fw, S.P1, S.r1(), s2);
            if (sb) CK_CHECK(hipEventRecord(c->sev[3], sb));
        };
        if (sb) {
            CK_CHECK(hipEventRecord(c->sev[0], st));
            CK_CHECK(hipStreamWaitEvent(sb, c->sev[0], 0));
        } else {
            side(st);
        }
        run_gemm(c, S, 3, st);  // W_mbej += 1/2 t2 <mn||ef>, written split
        if (sb) {
            side(sb);
            CK_CHECK(hipStreamWaitEvent(st, c->sev[2], 0));
        }
        run_gemm(c, S, 4, st);  // X += t2 W_mbej
        if (sb) CK_CHECK(hipStreamWaitEvent(st, c->sev[1], 0));
        run_gemm(c, S, 1, st);  // both ladders on canonical pairs, into Lp
        ck::launch_assemble_r2_pack(s, S.pairs(), S.X, S.Lp, S.r2c, S.npart, st);
        if (sb) CK_CHECK(hipStreamWaitEvent(st, c->sev[3], 0));
    }
    stage_end(c, all, st);
}

// every write of the amplitudes other than the mixed DIIS extrapolation
void amplitudes_changed(System &S) { S.sp_ok = S.e_ok = false; }

// a new trajectory (new inputs or amplitudes from the caller): empty DIIS history
void reset_iteration(System &S) {
    S.diis_reset = true;
    S.converged = false;
    S.rn_ref = INFINITY;
    S.stall = 0;
}

__global__ void k_copy_scalar(const double *src, double *dst) { *dst = *src; }

// ||R||^2 into S.redout[0] after residual_device (the mixed assembly left partial sums)
void launch_norm(System &S, hipStream_t st) {
    if (S.mixed) ck::launch_norm_pack(S.d, S.pairs(), S.npart, S.r1(), S.redout, st);
    else ck::launch_norm2(S.d, S.r1(), S.r2(), S.red, S.redout, st);
}

// The padding of the packed W_mnij and dressed <ab||ef> (pk_A, pk_B) is never written by
// their producers and must read as zero in the family's storage.  A 64-byte chunk holds the
// same eight elements in split and complex64 storage but at different bytes, so an element
// written in the other storage (a change of storage, or a timing run of another form)
// leaves non-zero bytes in the padding elements of its chunk.  Clearing both buffers
// restores the padding; the next residual rewrites every other element.
void clear_packed(System &S, hipStream_t st) {
    const int64_t R = S.PV + S.PO;
    CK_CHECK(hipMemsetAsync(S.pk_A, 0, 4 * S.d.N * (int64_t)S.PO * R * sizeof(uint16_t), st));
    CK_CHECK(hipMemsetAsync(S.pk_B, 0, 4 * S.d.N * (int64_t)S.PV * R * sizeof(uint16_t), st));
}

// split forms of the static <oo||vv> class (full for the ring W product, packed for W_mnij),
// from its complex64 copy widened into X (a scratch buffer of the same size, rewritten by
// every residual)
void static_split(System &S, hipStream_t st) {
    ck::launch_to_c128(S.n2(), S.oovv_c, S.X, st);
    ck::launch_operand(S.n2(), S.X, S.sp_oovv, S.c64_ring(), st);
    ck::launch_oovv_pack(S.d, S.dkc, S.pairs(), S.X, S.pk_oovv, S.c64_lad(), st);
}

// The mixed path's integral classes (complex64 only) from complex128 values, the device
// generator's (host == nullptr) or the caller's: each class passes through X (N^3 o^2 v^2
// complex128 elements, scratch that every residual rewrites) a range at a time.  <ab||ef>
// is kept on the dblk blocks only, in their order.
void mixed_inputs(System &S, const double *const *host, hipStream_t st) {
    static const char *cls[6] = {"oooo", "ooov", "oovv", "ovvo", "ovvv", "vvvv"};
    const int64_t N = S.d.N, o = S.d.no, v = S.d.nv, N3 = N * N * N;
    const int64_t bsz[6] = {o * o * o * o, o * o * o * v, o * o * v * v, o * v * v * o, o * v * v * v, v * v * v * v};
    const int32_t *dblk = S.ptab.data() + S.dblk_off();
    cd *stage = S.X;
    const int64_t cap = S.n2();
    // elements c0 .. c0+len-1 of class i (of its kept blocks for <ab||ef>) into the stage
    auto fill = [&](int i, int64_t c0, int64_t len) {
        if (!host) {
            ck::launch_synth_eri_range(S.mesh, (int)o, (int)v, S.desc.seed, S.desc.eri_scale, cls[i],
                                       i == 5 ? S.dblk_dev() : nullptr, c0, len, stage, st);
            return;
        }
        for (int64_t c = c0; c < c0 + len;) {  // contiguous runs of the caller's array
            int64_t src = c, n = c0 + len - c;
            if (i == 5) {
                const int64_t off = c % bsz[5];
                src = (int64_t)dblk[c / bsz[5]] * bsz[5] + off;
                n = std::min(n, bsz[5] - off);
            }
            CK_CHECK(hipMemcpyAsync(stage + (c - c0), host[i] + 2 * src, n * sizeof(cd), hipMemcpyHostToDevice, st));
            c += n;
        }
    };
    // <oo||vv> and <ov||vo> are exactly the size of the stage
    fill(2, 0, cap);
    ck::launch_round_c64(cap, stage, S.oovv_c, st);
    ck::launch_swap_last2_c64(N3 * o * o, (int)v, stage, S.oovvT_c, st);
    fill(3, 0, cap);
    ck::launch_ovvo_transpose_c64(S.d, stage, S.ovvoT_c, st);
    ck::cf *const dst[6] = {S.oooo_c, S.ooov_c, nullptr, nullptr, S.ovvv_c, S.vvvv_c};
    for (int i : {0, 1, 4, 5}) {
        const int64_t total = (i == 5 ? (int64_t)S.ndblk : N3) * bsz[i];
        for (int64_t c0 = 0; c0 < total; c0 += cap) {
            const int64_t len = std::min(cap, total - c0);  // a multiple of v^2 for ovvv
            fill(i, c0, len);
            ck::launch_round_c64(len, stage, dst[i] + c0, st);
            if (i == 4) ck::launch_swap_last2_c64(len / (v * v), (int)v, stage, S.ovvvT_c + c0, st);
        }
    }
    static_split(S, st);
}

double read_scalar(ccsd_k_ctx *c, const double *dptr) {
    double h = 0.0;
    CK_CHECK(hipMemcpyAsync(&h, dptr, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    CK_CHECK(hipStreamSynchronize(c->stream));
    return h;
}

int check_ctx(ccsd_k_ctx *c, bool need_bound = true) {
    if (!c) return CCSD_K_EINVAL;
    if (c->failed) return fail(c, CCSD_K_ESTATE, "context is unusable after a device error: " + c->err);
    if (need_bound && !c->bound) return fail(c, CCSD_K_ESTATE, "no workspace bound");
    return CCSD_K_OK;
}

int check_sys(ccsd_k_ctx *c, int32_t sys, bool need_inputs = true) {
    int rc = check_ctx(c);
    if (rc) return rc;
    if (sys < 0 || sys >= (int32_t)c->sys.size()) return fail(c, CCSD_K_EINVAL, "system index out of range");
    if (need_inputs && !c->sys[sys].inputs)
        return fail(c, CCSD_K_ESTATE, "inputs of system " + std::to_string(sys) + " not set");
    return CCSD_K_OK;
}


}  // namespace

// ====================================================================== ABI bodies
namespace {

int impl_init(const ccsd_k_system *sys, int32_t n_sys, void *hip_stream, ccsd_k_ctx **out) {
    if (out) *out = nullptr;
    if (!sys || !out) return fail(nullptr, CCSD_K_EINVAL, "null argument");
    if (n_sys < 1 || n_sys > 4096) return fail(nullptr, CCSD_K_EINVAL, "n_sys must be in 1..4096");
    // owned here until the plan is complete: a failure below (an invalid system, or a host
    // allocation of the tables) frees it
    std::unique_ptr<ccsd_k_ctx> holder(new ccsd_k_ctx());
    ccsd_k_ctx *c = holder.get();
    c->stream = (hipStream_t)hip_stream;
    c->sys.resize(n_sys);
    for (int s = 0; s < n_sys; ++s) {
        const ccsd_k_system &d = sys[s];
        System &S = c->sys[s];
        S.desc = d;
        std::string id = "system " + std::to_string(s) + ": ";
        if (d.grid[0] < 1 || d.grid[1] < 1 || d.grid[2] < 1 || (int64_t)d.grid[0] * d.grid[1] * d.grid[2] > CK_MAX_NK) {
            return fail(nullptr, CCSD_K_EINVAL, id + "grid entries must be >= 1 with N_k <= " + std::to_string(CK_MAX_NK));
        }
        if (d.n_occ < 1 || d.n_vir < 1 || d.n_occ > 256 || d.n_vir > 256) {
            return fail(nullptr, CCSD_K_EINVAL, id + "n_occ and n_vir must be in 1..256");
        }
        if (d.precision != CCSD_K_PREC_FP64 && d.precision != CCSD_K_PREC_MIXED) {
            return fail(nullptr, CCSD_K_EINVAL, id + "unsupported precision");
        }
        S.mixed = d.precision == CCSD_K_PREC_MIXED;
        if (d.grouping != CCSD_K_GROUPING_STANDARD && d.grouping != CCSD_K_GROUPING_REARRANGED)
            return fail(nullptr, CCSD_K_EINVAL, id + "unknown grouping");
        if (d.grouping == CCSD_K_GROUPING_REARRANGED && S.mixed)
            return fail(nullptr, CCSD_K_EINVAL, id + "the rearranged hole-hole grouping runs on the FP64 path only");
        if (d.diis_space != 0 && (d.diis_space < 2 || d.diis_space > 16)) {
            return fail(nullptr, CCSD_K_EINVAL, id + "diis_space must be 0 or 2..16");
        }
        if (d.synthetic && !(d.eri_scale > 0.0 && std::isfinite(d.eri_scale))) {
            return fail(nullptr, CCSD_K_EINVAL, id + "eri_scale must be positive");
        }
        S.mesh = ck::Mesh{d.grid[0], d.grid[1], d.grid[2], d.grid[0] * d.grid[1] * d.grid[2]};
        S.d = ck::Dims{S.mesh.N, d.n_occ, d.n_vir};
        int64_t N = S.mesh.N;
        S.kc.resize(N * N * N);
        for (int a = 0; a < N; ++a)
            for (int b = 0; b < N; ++b)
                for (int k = 0; k < N; ++k) S.kc[((int64_t)a * N + b) * N + k] = kcons(S.mesh, a, b, k);
        build_tables(S);
        for (int i = 0; i < 5; ++i) S.tile[i] = ck::f64_default_tile(S.g[i].op.G, S.g[i].op.M, S.g[i].op.N);
    }
    *out = holder.release();
    return CCSD_K_OK;
}

int impl_workspace_bytes(const ccsd_k_ctx *ctx, uint64_t *bytes) {
    if (!ctx || !bytes) return CCSD_K_EINVAL;
    Carver cv{0, 0, false};
    for (auto &S : const_cast<ccsd_k_ctx *>(ctx)->sys) carve(S, cv);
    double *norms = nullptr;
    cv.take(norms, (int64_t)ctx->sys.size());
    *bytes = cv.off + 256;
    return CCSD_K_OK;
}

int impl_bind_workspace(ccsd_k_ctx *ctx, void *device_ptr, uint64_t bytes) {
    int rc = check_ctx(ctx, false);
    if (rc) return rc;
    if (ctx->bound) return fail(ctx, CCSD_K_ESTATE, "workspace already bound");
    if (!device_ptr || ((uintptr_t)device_ptr & 255)) return fail(ctx, CCSD_K_EINVAL, "workspace must be 256-byte aligned");
    uint64_t need = 0;
    ccsd_k_workspace_bytes(ctx, &need);
    if (bytes < need)
        return fail(ctx, CCSD_K_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
    try {
        Carver cv{(uintptr_t)device_ptr, 0, true};
        for (auto &S : ctx->sys) carve(S, cv);
        cv.take(ctx->dnorms, (int64_t)ctx->sys.size());
        for (auto &S : ctx->sys) {
            CK_CHECK(hipMemcpyAsync(S.dkc, S.kc.data(), S.kc.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
            CK_CHECK(hipMemcpyAsync(S.dtab, S.tables.data(), S.tables.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                                    ctx->stream));
            CK_CHECK(hipMemsetAsync(S.amp, 0, (S.n1() + S.n2()) * sizeof(cd), ctx->stream));
            amplitudes_changed(S);
            CK_CHECK(hipMemsetAsync(S.res, 0, (S.mixed ? S.n1() : S.n1() + S.n2()) * sizeof(cd), ctx->stream));
            if (S.mixed) CK_CHECK(hipMemsetAsync(S.r2c, 0, S.n2() * sizeof(ck::cf), ctx->stream));
            CK_CHECK(hipMemsetAsync(S.zeros, 0, 16 * sizeof(cd), ctx->stream));
            CK_CHECK(hipMemcpyAsync(S.dptab, S.ptab.data(), S.ptab.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                    ctx->stream));
            if (S.mixed) clear_packed(S, ctx->stream);
            bind_ops(S);
            if (S.desc.synthetic) {
                static const char *cls[6] = {"oooo", "ooov", "oovv", "ovvo", "ovvv", "vvvv"};
                ck::launch_synth_fock(S.mesh, S.d.no, S.d.nv, S.desc.seed, S.fock, ctx->stream);
                ck::launch_diag(S.d, S.fock, S.eo, S.ev, ctx->stream);
                if (S.mixed) {
                    mixed_inputs(S, nullptr, ctx->stream);
                } else {
                    for (int i = 0; i < 6; ++i)
                        ck::launch_synth_eri(S.mesh, S.d.no, S.d.nv, S.desc.seed, S.desc.eri_scale, cls[i], S.eri[i],
                                             ctx->stream);
                    ck::launch_static_copies(S.dev(), S.statics(), ctx->stream);
                }
                S.inputs = true;
            }
        }
        CK_CHECK(hipStreamSynchronize(ctx->stream));
    } catch (const ck::HipError &e) {
        return fail(ctx, CCSD_K_EDEVICE, e.what);
    }
    ctx->ws = (char *)device_ptr;
    ctx->ws_bytes = bytes;
    ctx->bound = true;
    return CCSD_K_OK;
}

int impl_set_inputs(ccsd_k_ctx *ctx, int32_t sys, const double *fock, const double *const eri[6]) {
    int rc = check_sys(ctx, sys, false);
    if (rc) return rc;
    if (!fock || !eri) return fail(ctx, CCSD_K_EINVAL, "null input");
    for (int i = 0; i < 6; ++i)
        if (!eri[i]) return fail(ctx, CCSD_K_EINVAL, "null integral class");
    System &S = ctx->sys[sys];
    const int64_t N = S.d.N, o = S.d.no, v = S.d.nv, n = o + v, N3 = N * N * N;
    const int64_t cls[6] = {o * o * o * o, o * o * o * v, o * o * v * v, o * v * v * o, o * v * v * v, v * v * v * v};
    // The update of Sec. 4.4 divides by D_i^a = f_ii - f_aa (same k) and by
    // D_ij^ab = f_ii + f_jj - f_aa - f_bb over every momentum-conserving block: all of them
    // must be finite and nonzero.  When every occupied energy lies below every virtual one
    // (the usual case) all denominators are negative; otherwise each is checked.
    std::vector<double> eo(N * o), ev(N * v);
    double omax = -INFINITY, vmin = INFINITY;
    for (int64_t k = 0; k < N; ++k) {
        for (int64_t i = 0; i < o; ++i) eo[k * o + i] = fock[2 * ((k * n + i) * n + i)];
        for (int64_t a = 0; a < v; ++a) ev[k * v + a] = fock[2 * ((k * n + o + a) * n + o + a)];
    }
    for (double e : eo) {
        if (!std::isfinite(e)) return fail(ctx, CCSD_K_EINVAL, "non-finite orbital energy");
        omax = std::max(omax, e);
    }
    for (double e : ev) {
        if (!std::isfinite(e)) return fail(ctx, CCSD_K_EINVAL, "non-finite orbital energy");
        vmin = std::min(vmin, e);
    }
    if (!(omax < vmin)) {
        for (int64_t k = 0; k < N; ++k)
            for (int64_t i = 0; i < o; ++i)
                for (int64_t a = 0; a < v; ++a)
                    if (eo[k * o + i] - ev[k * v + a] == 0.0)
                        return fail(ctx, CCSD_K_EINVAL, "orbital energies give a zero T1 denominator");
        for (int64_t ki = 0; ki < N; ++ki)
            for (int64_t kj = 0; kj < N; ++kj)
                for (int64_t ka = 0; ka < N; ++ka) {
                    const int64_t kb = S.kc[(ki * N + kj) * N + ka];
                    for (int64_t i = 0; i < o; ++i)
                        for (int64_t j = 0; j < o; ++j)
                            for (int64_t a = 0; a < v; ++a)
                                for (int64_t b = 0; b < v; ++b) {
                                    const double D = eo[ki * o + i] + eo[kj * o + j] - ev[ka * v + a] - ev[kb * v + b];
                                    if (D == 0.0 || !std::isfinite(D))
                                        return fail(ctx, CCSD_K_EINVAL, "orbital energies give a zero T2 denominator");
                                }
                }
    }
    try {
        CK_CHECK(hipMemcpyAsync(S.fock, fock, N * n * n * sizeof(cd), hipMemcpyHostToDevice, ctx->stream));
        ck::launch_diag(S.d, S.fock, S.eo, S.ev, ctx->stream);
        if (S.mixed) {
            mixed_inputs(S, eri, ctx->stream);
        } else {
            for (int i = 0; i < 6; ++i)
                CK_CHECK(hipMemcpyAsync(S.eri[i], eri[i], N3 * cls[i] * sizeof(cd), hipMemcpyHostToDevice, ctx->stream));
            ck::launch_static_copies(S.dev(), S.statics(), ctx->stream);
        }
        S.e_ok = false;
        CK_CHECK(hipStreamSynchronize(ctx->stream));
    } catch (const ck::HipError &e) {
        return fail(ctx, CCSD_K_EDEVICE, e.what);
    }
    S.inputs = true;
    reset_iteration(S);  // a DIIS history of another Hamiltonian would mislead the next iterate
    return CCSD_K_OK;
}

int impl_residual(ccsd_k_ctx *ctx, int32_t sys, const double *t1, const double *t2, double *r1, double *r2) {
    int rc = check_sys(ctx, sys);
    if (rc) return rc;
    System &S = ctx->sys[sys];
    try {
        if (t1) CK_CHECK(hipMemcpyAsync(S.t1(), t1, S.n1() * sizeof(cd), hipMemcpyHostToDevice, ctx->stream));
        if (t2) CK_CHECK(hipMemcpyAsync(S.t2(), t2, S.n2() * sizeof(cd), hipMemcpyHostToDevice, ctx->stream));
        if (t1 || t2) {
            amplitudes_changed(S);
            reset_iteration(S);  // the caller's amplitudes start a new trajectory
        }
        ensure_side(ctx);
        residual_device(ctx, S, ctx->stream);
        launch_norm(S, ctx->stream);
        S.rnorm = std::sqrt(read_scalar(ctx, S.redout));
        if (r1) CK_CHECK(hipMemcpyAsync(r1, S.r1(), S.n1() * sizeof(cd), hipMemcpyDeviceToHost, ctx->stream));
        std::vector<ck::cf> r2h;
        if (r2 && S.mixed) {
            r2h.resize(S.n2());
            CK_CHECK(hipMemcpyAsync(r2h.data(), S.r2c, S.n2() * sizeof(ck::cf), hipMemcpyDeviceToHost, ctx->stream));
        } else if (r2) {
            CK_CHECK(hipMemcpyAsync(r2, S.r2(), S.n2() * sizeof(cd), hipMemcpyDeviceToHost, ctx->stream));
        }
        CK_CHECK(hipStreamSynchronize(ctx->stream));
        for (size_t i = 0; i < r2h.size(); ++i) {  // widened to the caller's complex128
            r2[2 * i] = r2h[i].x;
            r2[2 * i + 1] = r2h[i].y;
        }
        collect_timing(ctx);
    } catch (const ck::HipError &e) {
        return fail(ctx, CCSD_K_EDEVICE, e.what);
    }
    if (!std::isfinite(S.rnorm)) return fail(ctx, CCSD_K_ENUMERIC, "non-finite residual norm");
    return CCSD_K_OK;
}

// One iteration of the systems in `active`: residual, norm (also copied to the context's
// norm array), and the update gated on that norm (plain substitution, or the DIIS update,
// its step and the extrapolation), enqueued on the context's stream and its lanes with no
// host decision in between, so that it can be captured once and replayed as a graph.
void enqueue_iteration(ccsd_k_ctx *c, const std::vector<System *> &active, double tol) {
    const std::vector<hipStream_t> ls = fork_lanes(c, active);
    for (size_t k = 0; k < active.size(); ++k) {
        System &S = *active[k];
        const hipStream_t st = ls[k];
        residual_device(c, S, st);
        launch_norm(S, st);
        hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, st, S.redout, c->dnorms + (&S - c->sys.data()));
        CK_CHECK(hipGetLastError());
        const ck::Gate gate{S.redout, tol};
        const ck::SysDev sd = S.dev();
        if (S.desc.diis_space == 0) {
            if (S.mixed) ck::launch_update(sd, S.t1(), S.t2(), S.r1(), S.r2c, nullptr, nullptr, gate, st);
            else ck::launch_update(sd, S.t1(), S.t2(), S.r1(), S.r2(), nullptr, nullptr, gate, st);
            continue;
        }
        std::vector<const cd *> src(S.dvec.begin(), S.dvec.end());
        if (S.mixed) {
            ck::launch_update_diis_pack(sd, S.pairs(), S.amp, S.res, S.r2c, S.derr32.data(), S.dvec.data(), S.diis(),
                                        gate, S.red, st);
            ck::launch_lincomb_packed(sd, S.pairs(), src.data(), S.diis(), gate, S.amp, S.sp_t2, S.c64_ring(), S.epart,
                                      st);
        } else {
            ck::launch_update_diis_pack(sd, S.pairs(), S.amp, S.res, S.r2(), S.derr.data(), S.dvec.data(), S.diis(),
                                        gate, S.red, st);
            ck::launch_lincomb_packed(sd, S.pairs(), src.data(), S.diis(), gate, S.amp, nullptr, false, nullptr, st);
        }
    }
    join_lanes(c, ls);
}

// What a captured iteration depends on beyond the buffers: the active set, each system's
// arithmetic forms, k chunk and whether its residual re-splits t2, and the tolerance.
std::vector<int64_t> iteration_signature(ccsd_k_ctx *c, double tol) {
    std::vector<int64_t> sig;
    int64_t tb;
    std::memcpy(&tb, &tol, sizeof tb);
    sig.push_back(tb);
    for (const System &S : c->sys) {
        sig.push_back(S.converged ? -1 : 1);
        for (int a : S.arith) sig.push_back(a);
        for (int t : S.tile) sig.push_back(t);
        sig.push_back(S.kchunk);
        sig.push_back(S.sp_ok ? 1 : 0);
    }
    return sig;
}

void drop_graph(ccsd_k_ctx *c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->gsig.clear();
}

int impl_iterate(ccsd_k_ctx *ctx, int32_t max_iter, double tol, int32_t *iters, double *max_rnorm) {
    int rc = check_ctx(ctx);
    if (rc) return rc;
    if (max_iter < 0 || !(tol >= 0.0)) return fail(ctx, CCSD_K_EINVAL, "bad max_iter or tol");
    for (size_t s = 0; s < ctx->sys.size(); ++s)
        if (!ctx->sys[s].inputs) return fail(ctx, CCSD_K_ESTATE, "inputs of system " + std::to_string(s) + " not set");
    int done = 0;
    bool numeric_error = false;
    std::vector<double> hn(ctx->sys.size(), 0.0);
    try {
        for (auto &S : ctx->sys) S.converged = false;
        ensure_side(ctx);  // before any capture
        for (int it = 0; it < max_iter; ++it) {
            std::vector<System *> active;
            for (auto &S : ctx->sys)
                if (!S.converged) active.push_back(&S);
            if (active.empty()) break;
            for (System *S : active)
                if (S->diis_reset) {  // outside any captured work
                    CK_CHECK(hipMemsetAsync(S->dstate, 0, 4 * sizeof(int32_t), ctx->stream));
                    S->diis_reset = false;
                }
            if (ctx->graphs && !ctx->timing && ctx->stream) {  // (the null stream cannot be captured)
                const std::vector<int64_t> sig = iteration_signature(ctx, tol);
                if (!ctx->gexec || sig != ctx->gsig) {
                    drop_graph(ctx);
                    if (active.size() > 1) {  // the lanes exist before the capture starts
                        const std::vector<hipStream_t> ls0 = fork_lanes(ctx, active);
                        join_lanes(ctx, ls0);
                    }
                    CK_CHECK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeRelaxed));
                    try {
                        enqueue_iteration(ctx, active, tol);
                    } catch (...) {
                        hipGraph_t g = nullptr;
                        (void)hipStreamEndCapture(ctx->stream, &g);
                        if (g) (void)hipGraphDestroy(g);
                        throw;
                    }
                    hipGraph_t g = nullptr;
                    CK_CHECK(hipStreamEndCapture(ctx->stream, &g));
                    const hipError_t ie = hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0);
                    (void)hipGraphDestroy(g);
                    CK_CHECK(ie);
                    ctx->gsig = sig;
                }
                CK_CHECK(hipGraphLaunch(ctx->gexec, ctx->stream));
            } else {
                enqueue_iteration(ctx, active, tol);
            }
            CK_CHECK(hipMemcpyAsync(hn.data(), ctx->dnorms, hn.size() * sizeof(double), hipMemcpyDeviceToHost,
                                    ctx->stream));
            CK_CHECK(hipStreamSynchronize(ctx->stream));
            done = it + 1;
            for (System *S : active) {
                S->rnorm = std::sqrt(hn[S - ctx->sys.data()]);
                if (!std::isfinite(S->rnorm)) numeric_error = true;
                if (S->rnorm < tol) {  // the gate closed on the device too: no update
                    S->converged = true;
                    if (S->mixed) S->sp_ok = true;
                    continue;
                }
                // the update ran: the extrapolation of the mixed path left the operand copy
                // of t2 and the energy partial sums of the new amplitudes
                if (S->mixed && S->desc.diis_space > 0) S->sp_ok = S->e_ok = true;
                else amplitudes_changed(*S);
                if (ctx->escalate) watch_stagnation(ctx, *S);
            }
            if (numeric_error) break;
            collect_timing(ctx);
        }
    } catch (const ck::HipError &e) {
        drop_graph(ctx);
        return fail(ctx, CCSD_K_EDEVICE, e.what);
    }
    double worst = 0.0;
    bool all = true;
    for (auto &S : ctx->sys) {
        worst = std::max(worst, S.rnorm);
        all = all && S.converged;
    }
    if (iters) *iters = done;
    if (max_rnorm) *max_rnorm = worst;
    if (numeric_error) return fail(ctx, CCSD_K_ENUMERIC, "non-finite residual norm");
    return all ? CCSD_K_OK : CCSD_K_NOT_CONVERGED;
}

int impl_residual_norm(ccsd_k_ctx *ctx, int32_t sys, double *rnorm) {
    int rc = check_sys(ctx, sys, false);
    if (rc) return rc;
    if (!rnorm) return CCSD_K_EINVAL;
    *rnorm = ctx->sys[sys].rnorm;
    return CCSD_K_OK;
}

int impl_energy(ccsd_k_ctx *ctx, int32_t sys, double *e_re, double *e_im) {
    int rc = check_sys(ctx, sys);
    if (rc) return rc;
    System &S = ctx->sys[sys];
    double e[2] = {0.0, 0.0};
    try {
        if (S.e_ok) ck::launch_energy_packed(S.d, S.pairs(), S.epart, S.redout, ctx->stream);
        else ck::launch_energy(S.dev(), S.t1(), S.t2(), S.red, S.redout, ctx->stream);
        CK_CHECK(hipMemcpyAsync(e, S.redout, 2 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        CK_CHECK(hipStreamSynchronize(ctx->stream));
    } catch (const ck::HipError &er) {
        return fail(ctx, CCSD_K_EDEVICE, er.what);
    }
    if (e_re) *e_re = e[0];
    if (e_im) *e_im = e[1];
    if (!std::isfinite(e[0]) || !std::isfinite(e[1])) return fail(ctx, CCSD_K_ENUMERIC, "non-finite energy");
    return CCSD_K_OK;
}

int impl_get_amplitudes(ccsd_k_ctx *ctx, int32_t sys, double *t1, double *t2) {
    int rc = check_sys(ctx, sys, false);
    if (rc) return rc;
    System &S = ctx->sys[sys];
    try {
        if (t1) CK_CHECK(hipMemcpyAsync(t1, S.t1(), S.n1() * sizeof(cd), hipMemcpyDeviceToHost, ctx->stream));
        if (t2) CK_CHECK(hipMemcpyAsync(t2, S.t2(), S.n2() * sizeof(cd), hipMemcpyDeviceToHost, ctx->stream));
        CK_CHECK(hipStreamSynchronize(ctx->stream));
    } catch (const ck::HipError &e) {
        return fail(ctx, CCSD_K_EDEVICE, e.what);
    }
    return CCSD_K_OK;
}

int impl_set_amplitudes(ccsd_k_ctx *ctx, int32_t sys, const double *t1, const double *t2) {
    int rc = check_sys(ctx, sys, false);
    if (rc) return rc;
    System &S = ctx->sys[sys];
    try {
        if (t1) CK_CHECK(hipMemcpyAsync(S.t1(), t1, S.n1() * sizeof(cd), hipMemcpyHostToDevice, ctx->stream));
        if (t2) CK_CHECK(hipMemcpyAsync(S.t2(), t2, S.n2() * sizeof(cd), hipMemcpyHostToDevice, ctx->stream));
        amplitudes_changed(S);
        CK_CHECK(hipStreamSynchronize(ctx->stream));
    } catch (const ck::HipError &e) {
        return fail(ctx, CCSD_K_EDEVICE, e.what);
    }
    reset_iteration(S);
    return CCSD_K_OK;
}

int impl_flops(const ccsd_k_ctx *ctx, int32_t sys, double *gemm_flops, double *other_flops) {
    if (!ctx || sys < 0 || sys >= (int32_t)ctx->sys.size()) return CCSD_K_EINVAL;
    const ck::Dims &d = ctx->sys[sys].d;
    double N = d.N, o = d.no, v = d.nv;
    double N4 = N * N * N * N;
    double macs = N4 * o * o * v * v * v * v      // particle-particle ladder
                  + 2.0 * N4 * o * o * o * o * v * v  // W_mnij build + hole-hole ladder
                  + 2.0 * N4 * o * o * o * v * v * v;  // ring W build + ring product
    // the rearranged hole-hole grouping applies t2 X-tilde and t2 Y-tilde separately
    if (ctx->sys[sys].rearranged()) macs += N4 * o * o * o * o * v * v;
    if (gemm_flops) *gemm_flops = 8.0 * macs;
    double N3 = N * N * N;
    double small = N3 * (o * v * v * v * v * 2.0     // T1 dressing of <ab||ef>
                         + o * o * v * v * (4.0 * (o + v))  // assembly
                         + 2.0 * o * o * o * v * v           // ring seeds
                         + o * o * v * v * (v + o))          // W_mbej seed
                  + N3 * N * (o * o * o * v * v + o * o * v * v * v) * 2.0;  // F and R1 sums
    if (other_flops) *other_flops = 8.0 * small;
    return CCSD_K_OK;
}

int impl_product_shape(const ccsd_k_ctx *ctx, int32_t sys, int32_t product, int64_t *G, int64_t *M, int64_t *N,
                         int64_t *K) {
    if (!ctx || sys < 0 || sys >= (int32_t)ctx->sys.size() || product < 0 || product > 4) return CCSD_K_EINVAL;
    const System &S = ctx->sys[sys];
    // product numbering of the timing stages: 0 pp-ladder, 1 hh-ladder, 2 W_mnij, 3 ring W, 4 ring
    static const int gi[5] = {1, 2, 0, 3, 4};
    const int i = gi[product];
    if (S.mixed && i == 2) {  // the hole-hole ladder runs inside the particle-particle product
        if (G) *G = 0;
        if (M) *M = 0;
        if (N) *N = 0;
        if (K) *K = 0;
        return CCSD_K_OK;
    }
    const ck::GemmOps<cd> &o = (S.mixed && i < 2 ? S.gp[i] : S.g[i]).op;
    if (G) *G = o.G;
    if (M) *M = o.M;
    if (N) *N = o.N;
    if (K) *K = o.K;
    return CCSD_K_OK;
}

// product numbering of the timing stages (0 pp-ladder, 1 hh-ladder, 2 W_mnij, 3 ring W,
// 4 ring) -> mixed product slot of S.sg
constexpr int kSlotOfProduct[5] = {1, 2, 0, 3, 4};

// Give product slot i the arithmetic form a; when its family's storage changes, the static
// operands of the family are converted again and the split copy of t2 is marked stale.
void apply_form(ccsd_k_ctx *c, System &S, int slot, int a) {
    const bool lad = S.c64_lad(), ring = S.c64_ring();
    S.arith[slot] = a;
    if (lad != S.c64_lad()) clear_packed(S, c->stream);
    if (lad != S.c64_lad() || ring != S.c64_ring()) {
        S.sp_ok = false;
        if (S.inputs) static_split(S, c->stream);
    }
}

int check_mixed_product(ccsd_k_ctx *ctx, int32_t sys, int32_t product) {
    int rc = check_sys(ctx, sys, false);
    if (rc) return rc;
    if (!ctx->sys[sys].mixed) return fail(ctx, CCSD_K_EINVAL, "arithmetic forms apply to mixed-precision systems");
    if (product < 0 || product > 4 || product == 1)
        return fail(ctx, CCSD_K_EINVAL, "product must be 0, 2, 3 or 4 (the hole-hole ladder runs inside product 0)");
    return CCSD_K_OK;
}

int impl_set_product_form(ccsd_k_ctx *ctx, int32_t sys, int32_t product, int32_t form) {
    int rc = check_mixed_product(ctx, sys, product);
    if (rc) return rc;
    if (form < 0 || form >= ck::ARITH_COUNT) return fail(ctx, CCSD_K_EINVAL, "form must be in 0..3");
    System &S = ctx->sys[sys];
    try {
        apply_form(ctx, S, kSlotOfProduct[product], form);
        CK_CHECK(hipStreamSynchronize(ctx->stream));
    } catch (const ck::HipError &e) {
        return fail(ctx, CCSD_K_EDEVICE, e.what);
    }
    return CCSD_K_OK;
}

int impl_get_product_form(const ccsd_k_ctx *cctx, int32_t sys, int32_t product, int32_t *form) {
    ccsd_k_ctx *ctx = const_cast<ccsd_k_ctx *>(cctx);
    int rc = check_mixed_product(ctx, sys, product);
    if (rc) return rc;
    if (!form) return fail(ctx, CCSD_K_EINVAL, "null form");
    *form = ctx->sys[sys].arith[kSlotOfProduct[product]];
    return CCSD_K_OK;
}

int check_fp64_product(ccsd_k_ctx *ctx, int32_t sys, int32_t product) {
    int rc = check_sys(ctx, sys, false);
    if (rc) return rc;
    if (ctx->sys[sys].mixed) return fail(ctx, CCSD_K_EINVAL, "tile shapes apply to FP64 systems");
    if (product < 0 || product > 4) return fail(ctx, CCSD_K_EINVAL, "product must be in 0..4");
    return CCSD_K_OK;
}

int impl_set_product_tile(ccsd_k_ctx *ctx, int32_t sys, int32_t product, int32_t tile) {
    int rc = check_fp64_product(ctx, sys, product);
    if (rc) return rc;
    if (tile < 0 || tile >= ck::F64_TILE_COUNT) return fail(ctx, CCSD_K_EINVAL, "tile must be in 0..3");
    ctx->sys[sys].tile[kSlotOfProduct[product]] = tile;
    return CCSD_K_OK;
}

int impl_get_product_tile(const ccsd_k_ctx *cctx, int32_t sys, int32_t product, int32_t *tile) {
    ccsd_k_ctx *ctx = const_cast<ccsd_k_ctx *>(cctx);
    int rc = check_fp64_product(ctx, sys, product);
    if (rc) return rc;
    if (!tile) return fail(ctx, CCSD_K_EINVAL, "null tile");
    *tile = ctx->sys[sys].tile[kSlotOfProduct[product]];
    return CCSD_K_OK;
}

// Average launch time (ms) of FP64 product slot i with tile shape t; its outputs (the
// W_mnij and W_mbej seeds, X, r2) are rewritten by the next residual before use.
double time_tile(ccsd_k_ctx *c, System &S, int slot, int t, int reps) {
    hipEvent_t e0, e1;
    CK_CHECK(hipEventCreate(&e0));
    CK_CHECK(hipEventCreate(&e1));
    float ms = 0.f;
    try {
        ck::gemm_f64_tile(S.g[slot].op, t, c->stream);  // warm-up
        CK_CHECK(hipEventRecord(e0, c->stream));
        for (int r = 0; r < reps; ++r) ck::gemm_f64_tile(S.g[slot].op, t, c->stream);
        CK_CHECK(hipEventRecord(e1, c->stream));
        CK_CHECK(hipEventSynchronize(e1));
        CK_CHECK(hipEventElapsedTime(&ms, e0, e1));
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return (double)ms / reps;
}

// FP64 system: the fastest tile shape per product (all shapes give the same result).
int autotune_tiles(ccsd_k_ctx *ctx, System &S, const char *cache_path, int32_t *forms, double *report) {
    static_assert(ck::F64_TILE_COUNT <= ck::ARITH_COUNT, "tile times share the record layout");
    ck::TuneRecord rec[5];
    try {
        CK_CHECK(hipStreamSynchronize(ctx->stream));
        const std::string dev = ck::device_key();
        for (int slot = 0; slot < 5; ++slot) {
            const ck::GemmOps<cd> &o = S.g[slot].op;
            const std::string key = "f64tile:" + ck::tune_key(dev, o.G, o.M, o.N, o.K, 0);
            if (ck::cache_lookup(cache_path, key, rec[slot])) continue;
            ck::TuneRecord r;
            for (int t = 0; t < ck::F64_TILE_COUNT; ++t) r.ms[t] = time_tile(ctx, S, slot, t, 3);
            rec[slot] = r;
            ck::cache_store(cache_path, key, r);
        }
        for (int slot = 0; slot < 5; ++slot) {
            int b = ck::F64_TILE_64x64;
            for (int t = 0; t < ck::F64_TILE_COUNT; ++t)
                if (rec[slot].ms[t] < rec[slot].ms[b]) b = t;
            S.tile[slot] = b;
        }
        amplitudes_changed(S);
        CK_CHECK(hipStreamSynchronize(ctx->stream));
        if (forms)
            for (int p = 0; p < 5; ++p) forms[p] = S.tile[kSlotOfProduct[p]];
        if (report)
            for (int p = 0; p < 5; ++p)
                for (int a = 0; a < ck::ARITH_COUNT; ++a) {
                    report[(p * ck::ARITH_COUNT + a) * 2] = a < ck::F64_TILE_COUNT ? rec[kSlotOfProduct[p]].ms[a] : 0.0;
                    report[(p * ck::ARITH_COUNT + a) * 2 + 1] = 0.0;
                }
    } catch (const ck::HipError &e) {
        return fail(ctx, CCSD_K_EDEVICE, e.what);
    }
    return CCSD_K_OK;
}

// Average launch time (ms) of product slot i in arithmetic form a on the system's own
// operands and tables.  Timing does not depend on the values; the outputs it overwrites
// (W_mnij / W_mbej operands, Lp, X) are all recomputed by the next residual before use.
double time_form(ccsd_k_ctx *c, System &S, int slot, int a, int reps) {
    hipEvent_t e0, e1;
    CK_CHECK(hipEventCreate(&e0));
    CK_CHECK(hipEventCreate(&e1));
    float ms = 0.f;
    try {
        auto launch = [&] {
            if (ck::arith_c64(a)) ck::gemm_c64(S.sg[slot], a, c->stream);
            else ck::gemm_split(S.sg[slot], c->stream);
        };
        launch();  // warm-up
        CK_CHECK(hipEventRecord(e0, c->stream));
        for (int r = 0; r < reps; ++r) launch();
        CK_CHECK(hipEventRecord(e1, c->stream));
        CK_CHECK(hipEventSynchronize(e1));
        CK_CHECK(hipEventElapsedTime(&ms, e0, e1));
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return (double)ms / reps;
}

// Choose the arithmetic form of every mixed product of system sys: the fastest choice whose
// measured product error is within budget.  A family (ladder: slots 0, 1; ring: 3, 4) runs
// either all on split storage (every product PRESPLIT2) or all on complex64 storage (each
// product any of SPLIT2, SPLIT3, FP32); the faster admissible option wins.  With no
// admissible option the family takes, per product, the most accurate form.
int impl_autotune(ccsd_k_ctx *ctx, int32_t sys, double budget, const char *cache_path, int32_t *forms,
                  double *report) {
    int rc = check_sys(ctx, sys, false);
    if (rc) return rc;
    System &S = ctx->sys[sys];
    if (!(budget > 0.0)) return fail(ctx, CCSD_K_EINVAL, "budget must be positive");
    if (!S.mixed) return autotune_tiles(ctx, S, cache_path, forms, report);
    static const int slots[4] = {0, 1, 3, 4};  // W_mnij, ladders, W_mbej, ring
    ck::TuneRecord rec[5];
    try {
        CK_CHECK(hipStreamSynchronize(ctx->stream));
        const std::string dev = ck::device_key();
        for (int slot : slots) {
            const ck::SplitOps &o = S.sg[slot];
            const std::string key = ck::tune_key(dev, o.G, o.M, o.N, o.K, o.fast);
            if (ck::cache_lookup(cache_path, key, rec[slot])) continue;
            ck::TuneRecord r;
            for (int a = 0; a < ck::ARITH_COUNT; ++a) r.ms[a] = time_form(ctx, S, slot, a, 3);
            const std::vector<double> e =
                ck::form_errors(std::min(o.M, 256), std::min(o.N, 256), o.K, 1911 + slot, ctx->stream);
            for (int a = 0; a < ck::ARITH_COUNT; ++a) r.err[a] = e[a];
            rec[slot] = r;
            ck::cache_store(cache_path, key, r);
        }
        int choice[5];
        for (int fam = 0; fam < 2; ++fam) {
            const int s0 = slots[2 * fam], s1 = slots[2 * fam + 1];
            double t_split = -1.0, t_c64 = 0.0;
            bool c64_ok = true;
            if (rec[s0].err[0] <= budget && rec[s1].err[0] <= budget) t_split = rec[s0].ms[0] + rec[s1].ms[0];
            int best[2];
            for (int u = 0; u < 2; ++u) {
                const ck::TuneRecord &r = rec[u ? s1 : s0];
                int b = -1;
                for (int a = 1; a < ck::ARITH_COUNT; ++a)
                    if (r.err[a] <= budget && (b < 0 || r.ms[a] < r.ms[b])) b = a;
                if (b < 0) {  // nothing within budget: the most accurate form
                    c64_ok = false;
                    b = 1;
                    for (int a = 2; a < ck::ARITH_COUNT; ++a)
                        if (r.err[a] < r.err[b]) b = a;
                }
                best[u] = b;
                t_c64 += r.ms[b];
            }
            if (t_split >= 0.0 && (!c64_ok || t_split <= t_c64)) {
                choice[s0] = choice[s1] = ck::ARITH_PRESPLIT2;
            } else {
                choice[s0] = best[0];
                choice[s1] = best[1];
            }
        }
        // the timing runs left stale operands, and outputs written in the other storage:
        // recompute them from the amplitudes, with the packed padding cleared
        amplitudes_changed(S);
        clear_packed(S, ctx->stream);
        for (int slot : slots) S.arith[slot] = choice[slot];
        if (S.inputs) static_split(S, ctx->stream);
        CK_CHECK(hipStreamSynchronize(ctx->stream));
        if (forms)
            for (int p = 0; p < 5; ++p) forms[p] = p == 1 ? -1 : S.arith[kSlotOfProduct[p]];
        if (report)
            for (int p = 0; p < 5; ++p)
                for (int a = 0; a < ck::ARITH_COUNT; ++a) {
                    const bool none = p == 1;
                    report[(p * ck::ARITH_COUNT + a) * 2] = none ? 0.0 : rec[kSlotOfProduct[p]].ms[a];
                    report[(p * ck::ARITH_COUNT + a) * 2 + 1] = none ? 0.0 : rec[kSlotOfProduct[p]].err[a];
                }
    } catch (const ck::HipError &e) {
        return fail(ctx, CCSD_K_EDEVICE, e.what);
    }
    return CCSD_K_OK;
}

int impl_set_graphs(ccsd_k_ctx *ctx, int32_t enable) {
    int rc = check_ctx(ctx, false);
    if (rc) return rc;
    ctx->graphs = enable != 0;
    if (!ctx->graphs) drop_graph(ctx);
    return CCSD_K_OK;
}

int impl_set_overlap(ccsd_k_ctx *ctx, int32_t enable) {
    int rc = check_ctx(ctx, false);
    if (rc) return rc;
    ctx->overlap = enable != 0;
    drop_graph(ctx);  // a captured iteration holds the other form
    return CCSD_K_OK;
}

int impl_set_escalation(ccsd_k_ctx *ctx, int32_t enable) {
    int rc = check_ctx(ctx, false);
    if (rc) return rc;
    ctx->escalate = enable != 0;
    return CCSD_K_OK;
}

int impl_timing(ccsd_k_ctx *ctx, int32_t enable) {
    if (!ctx) return CCSD_K_EINVAL;
    try {
        collect_timing(ctx);
    } catch (const ck::HipError &e) {
        return fail(ctx, CCSD_K_EDEVICE, e.what);
    }
    ctx->timing = enable != 0;
    for (int i = 0; i < ST_COUNT; ++i) {
        ctx->stage_ms[i] = 0.0;
        ctx->stage_n[i] = 0;
    }
    return CCSD_K_OK;
}

int impl_timing_get(ccsd_k_ctx *ctx, int32_t stage, double *total_ms, int64_t *launches) {
    if (!ctx || stage < 0 || stage >= ST_COUNT) return CCSD_K_EINVAL;
    try {
        collect_timing(ctx);
    } catch (const ck::HipError &e) {
        return fail(ctx, CCSD_K_EDEVICE, e.what);
    }
    if (total_ms) *total_ms = ctx->stage_ms[stage];
    if (launches) *launches = ctx->stage_n[stage];
    return CCSD_K_OK;
}

int impl_debug_zgemm(int32_t G, int32_t M, int32_t N, int32_t K, const double *A, const double *B, double *C,
                       int32_t reference) {
    if (G < 1 || M < 1 || N < 1 || K < 0 || !A || !B || !C) return fail(nullptr, CCSD_K_EINVAL, "bad gemm arguments");
    std::vector<int64_t> tab;
    size_t o_arow = tab.size();
    for (int g = 0; g < G; ++g)
        for (int m = 0; m < M; ++m) tab.push_back(((int64_t)g * M + m) * K);
    size_t o_k = tab.size();
    for (int g = 0; g < G; ++g)
        for (int k = 0; k < K; ++k) tab.push_back(k);
    size_t o_bcol = tab.size();
    for (int g = 0; g < G; ++g)
        for (int n = 0; n < N; ++n) tab.push_back(((int64_t)g * N + n) * K);
    size_t o_crow = tab.size();
    for (int g = 0; g < G; ++g)
        for (int m = 0; m < M; ++m) tab.push_back(((int64_t)g * M + m) * N);
    size_t o_ccol = tab.size();
    for (int g = 0; g < G; ++g)
        for (int n = 0; n < N; ++n) tab.push_back(n);
    const size_t na = (size_t)G * M * K, nb = (size_t)G * N * K, nc = (size_t)G * M * N;
    cd *dA = nullptr, *dB = nullptr, *dC = nullptr, *dZ = nullptr;
    int64_t *dT = nullptr;
    int rc = CCSD_K_OK;
    try {
        CK_CHECK(hipMalloc(&dA, std::max<size_t>(na, 1) * sizeof(cd)));
        CK_CHECK(hipMalloc(&dB, std::max<size_t>(nb, 1) * sizeof(cd)));
        CK_CHECK(hipMalloc(&dC, nc * sizeof(cd)));
        CK_CHECK(hipMalloc(&dT, tab.size() * sizeof(int64_t)));
        CK_CHECK(hipMalloc(&dZ, 16 * sizeof(cd)));
        CK_CHECK(hipMemset(dZ, 0, 16 * sizeof(cd)));
        CK_CHECK(hipMemcpy(dA, A, na * sizeof(cd), hipMemcpyHostToDevice));
        CK_CHECK(hipMemcpy(dB, B, nb * sizeof(cd), hipMemcpyHostToDevice));
        CK_CHECK(hipMemcpy(dT, tab.data(), tab.size() * sizeof(int64_t), hipMemcpyHostToDevice));
        CK_CHECK(hipMemset(dC, 0, nc * sizeof(cd)));
        ck::GemmOps<cd> op{};
        op.A = dA; op.B = dB; op.C = dC; op.zeros = dZ;
        op.a_row = dT + o_arow; op.a_k = dT + o_k; op.b_col = dT + o_bcol; op.b_k = dT + o_k;
        op.c_row = dT + o_crow; op.c_col = dT + o_ccol;
        op.G = G; op.M = M; op.N = N; op.K = K; op.alpha = 1.0; op.beta = 0.0;
        if (reference == 1) {
            ck::gemm_f64_reference(op, nullptr);
        } else if (reference == 2) {
            // split-BF16 operands of A and B, product on the bf16 MFMA kernel
            auto padded = [](int64_t n) { return (n + 63) / 64 * 64; };
            int64_t pa = padded((int64_t)na), pb = padded((int64_t)nb);
            uint16_t *sA = nullptr, *sB = nullptr;
            CK_CHECK(hipMalloc(&sA, 4 * pa * sizeof(uint16_t)));
            CK_CHECK(hipMalloc(&sB, 4 * pb * sizeof(uint16_t)));
            ck::launch_split((int64_t)na, dA, sA, nullptr);
            ck::launch_split((int64_t)nb, dB, sB, nullptr);
            ck::SplitOps so{};
            so.A = sA; so.B = sB; so.C = dC;
            so.zeros = reinterpret_cast<const uint16_t *>(dZ);
            so.a_row = op.a_row; so.a_k = op.a_k; so.b_col = op.b_col; so.b_k = op.b_k;
            so.c_row = op.c_row; so.c_col = op.c_col;
            so.G = G; so.M = M; so.N = N; so.K = K; so.alpha = 1.0; so.beta = 0.0;
            so.fast = (K % 8 == 0) ? 1 : 0;
            ck::gemm_split(so, nullptr);
            CK_CHECK(hipDeviceSynchronize());
            (void)hipFree(sA);
            (void)hipFree(sB);
        } else if (reference >= 3 && reference <= 5) {
            // complex64 operands, product in the arithmetic form reference - 2 (split-BF16 with
            // two or three terms, or FP32 MFMA)
            auto padded = [](int64_t n) { return (n + 63) / 64 * 64; };
            int64_t pa = padded((int64_t)na), pb = padded((int64_t)nb);
            ck::cf *cA = nullptr, *cB = nullptr;
            CK_CHECK(hipMalloc(&cA, pa * sizeof(ck::cf)));
            CK_CHECK(hipMalloc(&cB, pb * sizeof(ck::cf)));
            ck::launch_to_c64((int64_t)na, dA, cA, nullptr);
            ck::launch_to_c64((int64_t)nb, dB, cB, nullptr);
            ck::SplitOps so{};
            so.A = reinterpret_cast<const uint16_t *>(cA); so.B = reinterpret_cast<const uint16_t *>(cB); so.C = dC;
            so.zeros = reinterpret_cast<const uint16_t *>(dZ);
            so.a_row = op.a_row; so.a_k = op.a_k; so.b_col = op.b_col; so.b_k = op.b_k;
            so.c_row = op.c_row; so.c_col = op.c_col;
            so.G = G; so.M = M; so.N = N; so.K = K; so.alpha = 1.0; so.beta = 0.0;
            so.fast = (K % 8 == 0) ? 1 : 0;
            ck::gemm_c64(so, reference - 2, nullptr);
            CK_CHECK(hipDeviceSynchronize());
            (void)hipFree(cA);
            (void)hipFree(cB);
        } else if (reference >= 23 && reference <= 25) {
            // complex64 operands, arithmetic form reference - 22, summed in FP64 over 64-k
            // chunks in one launch
            auto padded = [](int64_t n) { return (n + 63) / 64 * 64; };
            int64_t pa = padded((int64_t)na), pb = padded((int64_t)nb);
            ck::cf *cA = nullptr, *cB = nullptr;
            CK_CHECK(hipMalloc(&cA, pa * sizeof(ck::cf)));
            CK_CHECK(hipMalloc(&cB, pb * sizeof(ck::cf)));
            ck::launch_to_c64((int64_t)na, dA, cA, nullptr);
            ck::launch_to_c64((int64_t)nb, dB, cB, nullptr);
            ck::SplitOps so{};
            so.A = reinterpret_cast<const uint16_t *>(cA); so.B = reinterpret_cast<const uint16_t *>(cB); so.C = dC;
            so.zeros = reinterpret_cast<const uint16_t *>(dZ);
            so.a_row = op.a_row; so.a_k = op.a_k; so.b_col = op.b_col; so.b_k = op.b_k;
            so.c_row = op.c_row; so.c_col = op.c_col;
            so.G = G; so.M = M; so.N = N; so.K = K; so.alpha = 1.0; so.beta = 0.0;
            so.fast = (K % 8 == 0) ? 1 : 0;
            ck::gemm_c64_chunked(so, reference - 22, 64, nullptr);
            CK_CHECK(hipDeviceSynchronize());
            (void)hipFree(cA);
            (void)hipFree(cB);
        } else if (reference >= 10 && reference < 10 + ck::F64_TILE_COUNT) {
            ck::gemm_f64_tile(op, reference - 10, nullptr);  // the FP64 kernel in one tile shape
        } else {
            ck::gemm_f64(op, nullptr);
        }
        CK_CHECK(hipDeviceSynchronize());
        CK_CHECK(hipMemcpy(C, dC, nc * sizeof(cd), hipMemcpyDeviceToHost));
    } catch (const ck::HipError &e) {
        rc = fail(nullptr, CCSD_K_EDEVICE, e.what);
    }
    (void)hipFree(dA);
    (void)hipFree(dB);
    (void)hipFree(dC);
    (void)hipFree(dT);
    (void)hipFree(dZ);
    return rc;
}


// Every ABI entry runs inside this guard: no C++ exception crosses the C ABI.  Device
// errors surface as ck::HipError (EDEVICE), host allocation failures as std::bad_alloc.
template <class F>
int guarded(ccsd_k_ctx *c, F &&f) {
    try {
        return f();
    } catch (const ck::HipError &e) {
        return fail(c, CCSD_K_EDEVICE, e.what);
    } catch (const std::bad_alloc &) {
        return fail(c, CCSD_K_ENOMEM, "host memory allocation failed");
    } catch (const std::exception &e) {
        return fail(c, CCSD_K_EINVAL, std::string("internal error: ") + e.what());
    } catch (...) {
        return fail(c, CCSD_K_EINVAL, "unknown internal error");
    }
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

int ccsd_k_init(const ccsd_k_system *sys, int32_t n_sys, void *hip_stream, ccsd_k_ctx **out) {
    return guarded(nullptr, [&] { return impl_init(sys, n_sys, hip_stream, out); });
}

int ccsd_k_workspace_bytes(const ccsd_k_ctx *ctx, uint64_t *bytes) {
    return guarded(const_cast<ccsd_k_ctx *>(ctx), [&] { return impl_workspace_bytes(ctx, bytes); });
}

int ccsd_k_bind_workspace(ccsd_k_ctx *ctx, void *device_ptr, uint64_t bytes) {
    return guarded(ctx, [&] { return impl_bind_workspace(ctx, device_ptr, bytes); });
}

int ccsd_k_set_inputs(ccsd_k_ctx *ctx, int32_t sys, const double *fock, const double *const eri[6]) {
    return guarded(ctx, [&] { return impl_set_inputs(ctx, sys, fock, eri); });
}

int ccsd_k_residual(ccsd_k_ctx *ctx, int32_t sys, const double *t1, const double *t2, double *r1, double *r2) {
    return guarded(ctx, [&] { return impl_residual(ctx, sys, t1, t2, r1, r2); });
}

int ccsd_k_iterate(ccsd_k_ctx *ctx, int32_t max_iter, double tol, int32_t *iters, double *max_rnorm) {
    return guarded(ctx, [&] { return impl_iterate(ctx, max_iter, tol, iters, max_rnorm); });
}

int ccsd_k_residual_norm(ccsd_k_ctx *ctx, int32_t sys, double *rnorm) {
    return guarded(ctx, [&] { return impl_residual_norm(ctx, sys, rnorm); });
}

int ccsd_k_energy(ccsd_k_ctx *ctx, int32_t sys, double *e_re, double *e_im) {
    return guarded(ctx, [&] { return impl_energy(ctx, sys, e_re, e_im); });
}

int ccsd_k_get_amplitudes(ccsd_k_ctx *ctx, int32_t sys, double *t1, double *t2) {
    return guarded(ctx, [&] { return impl_get_amplitudes(ctx, sys, t1, t2); });
}

int ccsd_k_set_amplitudes(ccsd_k_ctx *ctx, int32_t sys, const double *t1, const double *t2) {
    return guarded(ctx, [&] { return impl_set_amplitudes(ctx, sys, t1, t2); });
}

int ccsd_k_flops(const ccsd_k_ctx *ctx, int32_t sys, double *gemm_flops, double *other_flops) {
    return guarded(const_cast<ccsd_k_ctx *>(ctx), [&] { return impl_flops(ctx, sys, gemm_flops, other_flops); });
}

int ccsd_k_product_shape(const ccsd_k_ctx *ctx, int32_t sys, int32_t product, int64_t *G, int64_t *M, int64_t *N,
                         int64_t *K) {
    return guarded(const_cast<ccsd_k_ctx *>(ctx), [&] { return impl_product_shape(ctx, sys, product, G, M, N, K); });
}

int ccsd_k_set_product_form(ccsd_k_ctx *ctx, int32_t sys, int32_t product, int32_t form) {
    return guarded(ctx, [&] { return impl_set_product_form(ctx, sys, product, form); });
}

int ccsd_k_get_product_form(const ccsd_k_ctx *ctx, int32_t sys, int32_t product, int32_t *form) {
    return guarded(const_cast<ccsd_k_ctx *>(ctx), [&] { return impl_get_product_form(ctx, sys, product, form); });
}

int ccsd_k_set_product_tile(ccsd_k_ctx *ctx, int32_t sys, int32_t product, int32_t tile) {
    return guarded(ctx, [&] { return impl_set_product_tile(ctx, sys, product, tile); });
}

int ccsd_k_get_product_tile(const ccsd_k_ctx *ctx, int32_t sys, int32_t product, int32_t *tile) {
    return guarded(const_cast<ccsd_k_ctx *>(ctx), [&] { return impl_get_product_tile(ctx, sys, product, tile); });
}

int ccsd_k_autotune(ccsd_k_ctx *ctx, int32_t sys, double budget, const char *cache_path, int32_t *forms,
                    double *report) {
    return guarded(ctx, [&] { return impl_autotune(ctx, sys, budget, cache_path, forms, report); });
}

int ccsd_k_set_graphs(ccsd_k_ctx *ctx, int32_t enable) {
    return guarded(ctx, [&] { return impl_set_graphs(ctx, enable); });
}

int ccsd_k_set_overlap(ccsd_k_ctx *ctx, int32_t enable) {
    return guarded(ctx, [&] { return impl_set_overlap(ctx, enable); });
}

int ccsd_k_set_escalation(ccsd_k_ctx *ctx, int32_t enable) {
    return guarded(ctx, [&] { return impl_set_escalation(ctx, enable); });
}

int ccsd_k_timing(ccsd_k_ctx *ctx, int32_t enable) {
    return guarded(ctx, [&] { return impl_timing(ctx, enable); });
}

int ccsd_k_timing_get(ccsd_k_ctx *ctx, int32_t stage, double *total_ms, int64_t *launches) {
    return guarded(ctx, [&] { return impl_timing_get(ctx, stage, total_ms, launches); });
}

int ccsd_k_zgemm_noalloc(int32_t G, int32_t M, int32_t N, int32_t K, const double *A, const double *B, double *C,
                         int32_t variant, void *hip_stream) {
    return guarded(nullptr, [&] {
        std::string err;
        const int rc = ck::noalloc_zgemm(G, M, N, K, A, B, C, variant, (hipStream_t)hip_stream, err);
        if (rc == 0) return CCSD_K_OK;
        return fail(nullptr, rc == -1 ? CCSD_K_EINVAL : CCSD_K_EDEVICE, err);
    });
}

int ccsd_k_debug_zgemm(int32_t G, int32_t M, int32_t N, int32_t K, const double *A, const double *B, double *C,
                       int32_t reference) {
    return guarded(nullptr, [&] { return impl_debug_zgemm(G, M, N, K, A, B, C, reference); });
}

void ccsd_k_free(ccsd_k_ctx *ctx) {
    if (!ctx) return;
    drop_graph(ctx);
    if (!ctx->failed) {
        (void)hipStreamSynchronize(ctx->stream);
        for (auto &p : ctx->pending) ctx->pool.push_back(p);
        for (auto &p : ctx->pool) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
        for (hipStream_t st : ctx->lanes) (void)hipStreamSynchronize(st);
        if (ctx->side) (void)hipStreamSynchronize(ctx->side);
    }
    // after a device error the handles are still released (best effort, errors ignored)
    for (hipStream_t st : ctx->lanes) (void)hipStreamDestroy(st);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    for (hipEvent_t ev : ctx->sev)
        if (ev) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : ctx->joins) (void)hipEventDestroy(ev);
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    if (ctx->failed) {
        for (auto &p : ctx->pending) ctx->pool.push_back(p);
        for (auto &p : ctx->pool) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
    }
    delete ctx;
}

const char *ccsd_k_last_error(const ccsd_k_ctx *ctx) { return ctx ? ctx->err.c_str() : g_init_error.c_str(); }

}  // extern "C"
