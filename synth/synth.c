/*
 * Seeded synthetic inputs for periodic spin-orbital CCSD test systems.
 *
 * This file is input generation only: it holds none of the coupled-cluster
 * arithmetic.  It produces, for a Gamma-containing regular k-mesh,
 *   - a diagonal Fock matrix per k point,
 *   - antisymmetrized, Hermitian two-electron integrals <pq||rs> by
 *     occupied/virtual class, with k_s fixed by momentum conservation
 *     (k_p + k_q = k_r + k_s modulo a reciprocal lattice vector),
 *   - optional random test amplitudes.
 *
 * Recipe (every element independent of materialization order):
 *   stream state   s_tag = mix64(mix64(seed) ^ tag)
 *   n-th draw      h_n   = mix64(s_tag + (n + 1) * 0x9E3779B97F4A7C15)
 *                  (the n-th output of Steele-Lea-Flood splitmix64 started at s_tag)
 *   uniform        u     = ((h >> 11) + 0.5) * 2^-53            in (0, 1)
 *   raw integral   g(kp,kq,kr;p,q,r,s), counter L = ((((((kp*N+kq)*N+kr)*n+p)*n+q)*n+r)*n+s)
 *                  u1 = u(h_{2L}), u2 = u(h_{2L+1}), Box-Muller:
 *                  g = scale * sqrt(-2 ln u1) * (cos(2 pi u2) + i sin(2 pi u2))
 *   antisymmetrize A_pqrs = ((g_pqrs + g_qpsr) - (g_qprs + g_pqsr)) / 4
 *   Hermitize      H_pqrs = (A_pqrs + conj(A_rspq)) / 2
 *   Fock           f_pp(k) = -2 + 1.5 u (occupied) or 0.5 + 2.5 u (virtual),
 *                  u from draw k*n + p of stream tag 1; off-diagonal 0.
 * Tags: 1 Fock, 2 integrals, 3 batch shapes, 4 test T1, 5 test T2.
 * Orbital p of class 'o' is p, of class 'v' is n_occ + p, of class 'n' is p.
 * Arrays are complex128 interleaved (re, im), C order.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t synth_stream_state(uint64_t seed, uint64_t tag) { return mix64(mix64(seed) ^ tag); }

uint64_t synth_draw(uint64_t state, uint64_t n) { return mix64(state + (n + 1) * GOLDEN); }

double synth_uniform(uint64_t state, uint64_t n) {
    return ((double)(synth_draw(state, n) >> 11) + 0.5) * 0x1.0p-53;
}

typedef struct {
    int g[3];
    int N, n;
} mesh_t;

static mesh_t make_mesh(const int32_t grid[3], int n) {
    mesh_t m;
    m.g[0] = grid[0];
    m.g[1] = grid[1];
    m.g[2] = grid[2];
    m.N = grid[0] * grid[1] * grid[2];
    m.n = n;
    return m;
}

/* k_s = k_p + k_q - k_r, component-wise modulo the grid, C-order linear index. */
static inline int kconserve(const mesh_t *m, int kp, int kq, int kr) {
    int a[3], b[3], c[3], s = 0;
    int xp = kp, xq = kq, xr = kr;
    for (int d = 2; d >= 0; --d) {
        a[d] = xp % m->g[d]; xp /= m->g[d];
        b[d] = xq % m->g[d]; xq /= m->g[d];
        c[d] = xr % m->g[d]; xr /= m->g[d];
    }
    for (int d = 0; d < 3; ++d) {
        int v = (a[d] + b[d] - c[d]) % m->g[d];
        if (v < 0) v += m->g[d];
        s = s * m->g[d] + v;
    }
    return s;
}

int synth_kconserve(const int32_t grid[3], int kp, int kq, int kr) {
    mesh_t m = make_mesh(grid, 1);
    return kconserve(&m, kp, kq, kr);
}

static inline void raw_g(const mesh_t *m, uint64_t st, double scale, int kp, int kq, int kr,
                         int p, int q, int r, int s, double *re, double *im) {
    const uint64_t n = (uint64_t)m->n, N = (uint64_t)m->N;
    uint64_t L = ((((((uint64_t)kp * N + kq) * N + kr) * n + p) * n + q) * n + r) * n + s;
    double u1 = synth_uniform(st, 2 * L), u2 = synth_uniform(st, 2 * L + 1);
    double rad = sqrt(-2.0 * log(u1));
    double ph = 2.0 * M_PI * u2;
    *re = scale * rad * cos(ph);
    *im = scale * rad * sin(ph);
}

static inline void anti_A(const mesh_t *m, uint64_t st, double scale, int kp, int kq, int kr,
                          int p, int q, int r, int s, double *re, double *im) {
    int ks = kconserve(m, kp, kq, kr);
    double ar, ai, br, bi, cr, ci, dr, di;
    raw_g(m, st, scale, kp, kq, kr, p, q, r, s, &ar, &ai);
    raw_g(m, st, scale, kq, kp, kr, q, p, r, s, &br, &bi);
    raw_g(m, st, scale, kp, kq, ks, p, q, s, r, &cr, &ci);
    raw_g(m, st, scale, kq, kp, ks, q, p, s, r, &dr, &di);
    /* (a + d) - (b + c): the swapped combinations are exact negations in IEEE arithmetic */
    *re = 0.25 * ((ar + dr) - (br + cr));
    *im = 0.25 * ((ai + di) - (bi + ci));
}

/* One element of the physical integral H_pqrs (full orbital indices). */
void synth_eri_element(uint64_t seed, const int32_t grid[3], int n, double scale, int kp, int kq,
                       int kr, int p, int q, int r, int s, double out[2]) {
    mesh_t m = make_mesh(grid, n);
    uint64_t st = synth_stream_state(seed, 2);
    int ks = kconserve(&m, kp, kq, kr);
    double ar, ai, br, bi;
    anti_A(&m, st, scale, kp, kq, kr, p, q, r, s, &ar, &ai);
    anti_A(&m, st, scale, kr, ks, kp, r, s, p, q, &br, &bi);
    out[0] = 0.5 * (ar + br);
    out[1] = 0.5 * (ai - bi);
}

static int class_dim(char c, int no, int nv) { return c == 'o' ? no : (c == 'v' ? nv : no + nv); }
static int class_off(char c, int no) { return c == 'v' ? no : 0; }

/* One momentum block [kp,kq,kr] of class cls (4 chars of o/v/n): out[d0][d1][d2][d3] complex. */
static void eri_block(const mesh_t *m, uint64_t st, double scale, int no, int nv, const char *cls,
                      int kp, int kq, int kr, double *out) {
    int d[4], o[4];
    for (int t = 0; t < 4; ++t) {
        d[t] = class_dim(cls[t], no, nv);
        o[t] = class_off(cls[t], no);
    }
    int ks = kconserve(m, kp, kq, kr);
    size_t idx = 0;
    for (int p = 0; p < d[0]; ++p)
        for (int q = 0; q < d[1]; ++q)
            for (int r = 0; r < d[2]; ++r)
                for (int s = 0; s < d[3]; ++s, ++idx) {
                    int P = p + o[0], Q = q + o[1], R = r + o[2], S = s + o[3];
                    double ar, ai, br, bi;
                    anti_A(m, st, scale, kp, kq, kr, P, Q, R, S, &ar, &ai);
                    anti_A(m, st, scale, kr, ks, kp, R, S, P, Q, &br, &bi);
                    out[2 * idx] = 0.5 * (ar + br);
                    out[2 * idx + 1] = 0.5 * (ai - bi);
                }
}

int synth_eri_block(uint64_t seed, const int32_t grid[3], int no, int nv, double scale,
                    const char *cls, int kp, int kq, int kr, double *out) {
    if (strlen(cls) != 4) return -1;
    mesh_t m = make_mesh(grid, no + nv);
    eri_block(&m, synth_stream_state(seed, 2), scale, no, nv, cls, kp, kq, kr, out);
    return 0;
}

/* All blocks of a class: out[kp][kq][kr][d0][d1][d2][d3]. */
int synth_eri_class(uint64_t seed, const int32_t grid[3], int no, int nv, double scale,
                    const char *cls, double *out) {
    if (strlen(cls) != 4) return -1;
    mesh_t m = make_mesh(grid, no + nv);
    uint64_t st = synth_stream_state(seed, 2);
    size_t blk = 1;
    for (int t = 0; t < 4; ++t) blk *= (size_t)class_dim(cls[t], no, nv);
    long nblk = (long)m.N * m.N * m.N;
#pragma omp parallel for schedule(dynamic, 1)
    for (long b = 0; b < nblk; ++b) {
        int kp = (int)(b / ((long)m.N * m.N)), kq = (int)((b / m.N) % m.N), kr = (int)(b % m.N);
        eri_block(&m, st, scale, no, nv, cls, kp, kq, kr, out + 2 * blk * (size_t)b);
    }
    return 0;
}

/* Diagonal Fock: out[k][n][n] complex. */
int synth_fock(uint64_t seed, const int32_t grid[3], int no, int nv, double *out) {
    mesh_t m = make_mesh(grid, no + nv);
    uint64_t st = synth_stream_state(seed, 1);
    int n = no + nv;
    memset(out, 0, sizeof(double) * 2 * (size_t)m.N * n * n);
    for (int k = 0; k < m.N; ++k)
        for (int p = 0; p < n; ++p) {
            double u = synth_uniform(st, (uint64_t)k * n + p);
            out[2 * ((size_t)k * n * n + (size_t)p * n + p)] = p < no ? -2.0 + 1.5 * u : 0.5 + 2.5 * u;
        }
    return 0;
}

/* Uniform draws in (0,1) from stream tag, counters [0, count). */
int synth_uniforms(uint64_t seed, uint64_t tag, uint64_t count, double *out) {
    uint64_t st = synth_stream_state(seed, tag);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < (long)count; ++i) out[i] = synth_uniform(st, (uint64_t)i);
    return 0;
}

/*
 * Random test amplitudes of a given magnitude: t1[k][i][a] and t2[ki][kj][ka][i][j][a][b],
 * each element scale*(u-0.5 + i(u'-0.5)) before projection; t2 is then antisymmetrized in
 * (i,j) and (a,b) with momentum labels attached, so that t2 has the symmetry of the
 * amplitudes it stands for.
 */
static inline void raw_t2(const mesh_t *m, uint64_t st, int no, int nv, double scale, int ki,
                          int kj, int ka, int i, int j, int a, int b, double *re, double *im) {
    uint64_t N = (uint64_t)m->N;
    uint64_t L = ((((((uint64_t)ki * N + kj) * N + ka) * no + i) * no + j) * nv + a) * nv + b;
    *re = scale * (synth_uniform(st, 2 * L) - 0.5);
    *im = scale * (synth_uniform(st, 2 * L + 1) - 0.5);
}

int synth_test_amplitudes(uint64_t seed, const int32_t grid[3], int no, int nv, double scale,
                          double *t1, double *t2) {
    mesh_t m = make_mesh(grid, no + nv);
    uint64_t s1 = synth_stream_state(seed, 4), s2 = synth_stream_state(seed, 5);
    int N = m.N;
    if (t1)
        for (long idx = 0; idx < (long)N * no * nv; ++idx) {
            t1[2 * idx] = scale * (synth_uniform(s1, 2 * (uint64_t)idx) - 0.5);
            t1[2 * idx + 1] = scale * (synth_uniform(s1, 2 * (uint64_t)idx + 1) - 0.5);
        }
    if (!t2) return 0;
    size_t blk = (size_t)no * no * nv * nv;
    long nblk = (long)N * N * N;
#pragma omp parallel for schedule(dynamic, 1)
    for (long bk = 0; bk < nblk; ++bk) {
        int ki = (int)(bk / ((long)N * N)), kj = (int)((bk / N) % N), ka = (int)(bk % N);
        int kb = kconserve(&m, ki, kj, ka);
        double *o = t2 + 2 * blk * (size_t)bk;
        size_t idx = 0;
        for (int i = 0; i < no; ++i)
            for (int j = 0; j < no; ++j)
                for (int a = 0; a < nv; ++a)
                    for (int b = 0; b < nv; ++b, ++idx) {
                        double r0, i0, r1, i1, r2, i2, r3, i3;
                        raw_t2(&m, s2, no, nv, scale, ki, kj, ka, i, j, a, b, &r0, &i0);
                        raw_t2(&m, s2, no, nv, scale, kj, ki, ka, j, i, a, b, &r1, &i1);
                        raw_t2(&m, s2, no, nv, scale, ki, kj, kb, i, j, b, a, &r2, &i2);
                        raw_t2(&m, s2, no, nv, scale, kj, ki, kb, j, i, b, a, &r3, &i3);
                        o[2 * idx] = 0.25 * ((r0 + r3) - (r1 + r2));
                        o[2 * idx + 1] = 0.25 * ((i0 + i3) - (i1 + i2));
                    }
    }
    return 0;
}
