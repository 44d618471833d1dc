// Host plan builder: grid, y operators, x/z eigenbases, device blob image.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <new>

#include "ibs_internal.h"
#include "multigrid.h"

namespace ibs {

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// The FP64 transforms fold the real Fourier basis when the half length is a
// whole number of 16-blocks.
bool can_fold(int n) { return n % 32 == 0; }

// Row counts the cyclic tridiagonal is instantiated for (periodic y): the
// P chunks of M rows hold the system exactly, n = P M (k_tridiag_cyc.hip).
bool cyclic_rows_supported(int n)
{
    switch (n) {
    case 48: case 64: case 80: case 96: case 128: case 160: case 192: case 256: case 320: case 384:
    case 512: return true;
    default: return false;
    }
}

// Real orthonormal Fourier basis of the periodic 3-point second difference
// (its eigenvectors; eigenvalues are minus the modified wavenumber squared,
// -(2/h^2)(1 - cos(kappa h)) = -(4/h^2) sin^2(pi k / N), Appendix A).
// Column order: a = 0 constant; a = 1..N/2-1 cosines of wavenumber a;
// a = N/2 the alternating mode; a = N/2+1..N-1 sines of wavenumber a - N/2.
// Angles are reduced exactly, 2 pi ((k i) mod N) / N, and evaluated in long
// double.  Q is row-major: Q[i*N + a] = mode a at grid index i.
static void fourier_basis(int N, double h, std::vector<double> &Q, std::vector<double> &lam)
{
    Q.assign(size_t(N) * N, 0.0);
    lam.assign(N, 0.0);
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double s0 = 1.0L / std::sqrt((long double)N);
    const long double s1 = std::sqrt(2.0L / (long double)N);
    const int half = N / 2;
    // only N distinct angles 2 pi m / N occur (m = k i mod N)
    std::vector<long double> ct(N), st(N);
    for (int m = 0; m < N; ++m) {
        const long double th = 2.0L * pi * (long double)m / (long double)N;
        ct[m] = std::cos(th);
        st[m] = std::sin(th);
    }
    for (int a = 0; a < N; ++a) {
        int k = (a <= half) ? a : a - half;
        long double sk = std::sin(pi * (long double)k / (long double)N);
        lam[a] = (double)(-(4.0L / ((long double)h * h)) * sk * sk);
        for (int i = 0; i < N; ++i) {
            const int m = (int)(((long long)k * i) % N);
            long double v;
            if (a == 0) v = s0;
            else if (a < half) v = s1 * ct[m];
            else if (a == half) v = (i % 2 == 0) ? s0 : -s0;
            else v = s1 * st[m];
            Q[size_t(i) * N + a] = (double)v;
        }
    }
}

// Orthonormal eigenbases of the wall-bounded 3-point second differences on
// n uniform cells of width h (x walls), each with its eigenvalues
// -(4/h^2) sin^2(pi a / (2n)):
//   XK_P, Neumann on cell centres:    cos(pi a (i + 1/2) / n), a = 0..n-1
//   XK_C, mirror Dirichlet, centres:  sin(pi a (i + 1/2) / n), a = 1..n
//                                     (column a - 1)
//   XK_F, Dirichlet on faces 1..n-1:  sin(pi a i / n), a = 1..n-1 (column
//                                     a); column 0 and row 0 (the wall slot)
//                                     zero, eigenvalue 0
// scaled to unit norm (sqrt(2/n), or sqrt(1/n) for the constant and the
// alternating columns).  Angles reduced exactly: every one is pi m / (2n)
// with m = (a (2i + 1)) mod 4n or 2 (a i mod 2n), evaluated in long double.
static void wall_basis(int n, double h, int xk, std::vector<double> &Q, std::vector<double> &lam)
{
    Q.assign(size_t(n) * n, 0.0);
    lam.assign(n, 0.0);
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<long double> cs(4 * n), sn(4 * n);
    for (int m = 0; m < 4 * n; ++m) {
        const long double th = pi * (long double)m / (2.0L * n);
        cs[m] = std::cos(th);
        sn[m] = std::sin(th);
    }
    const long double r1 = std::sqrt(1.0L / n), r2 = std::sqrt(2.0L / n);
    auto eig = [&](int a) {
        const long double sk = sn[a % (4 * n)];   // sin(pi a / (2n))
        return (double)(-(4.0L / ((long double)h * h)) * sk * sk);
    };
    for (int col = 0; col < n; ++col) {
        int a = col;
        if (xk == XK_C) a = col + 1;
        if (xk == XK_F && col == 0) continue;   // the wall slot
        lam[col] = eig(a);
        for (int i = 0; i < n; ++i) {
            long double v;
            if (xk == XK_F) {
                v = r2 * sn[(2LL * (((long long)a * i) % (2 * n))) % (4 * n)];
            } else {
                const int m = (int)(((long long)a * (2 * i + 1)) % (4 * n));
                const long double scale = (a == 0 || a == n) ? r1 : r2;
                v = scale * (xk == XK_P ? cs[m] : sn[m]);
            }
            Q[size_t(i) * n + col] = (double)v;
        }
    }
}

// Eigenpairs of a real symmetric tridiagonal matrix (diagonal d[0..m-1],
// off-diagonal e[i] coupling rows i and i+1), by the implicit QL iteration
// with Wilkinson's shift (Bowdler, Martin, Reinsch and Wilkinson, 1968):
// each sweep chases the shifted QL bulge up from the first negligible
// off-diagonal with plane rotations, which are accumulated into V (m x m,
// row-major, V[i*m + a] = component i of eigenvector a).  Runs in long
// double, so the eigenvalues carry absolute errors near 1e-19 ||T||: the
// smallest ones (the modes that matter most to a solve) stay accurate to
// about 1e-15 relative at the grid sizes served.  On return d holds the
// eigenvalues (unsorted).  Returns false if some eigenvalue needs more
// than 60 sweeps.
static bool tridiag_eigen(int m, std::vector<long double> &d, std::vector<long double> e,
                          std::vector<long double> &V)
{
    V.assign(size_t(m) * m, 0.0L);
    for (int i = 0; i < m; ++i) V[size_t(i) * m + i] = 1.0L;
    e.resize(m, 0.0L);
    e[m - 1] = 0.0L;
    const long double eps = std::numeric_limits<long double>::epsilon();
    for (int l = 0; l < m; ++l) {
        for (int sweep = 0;; ++sweep) {
            int k = l;   // first negligible coupling at or after l
            while (k + 1 < m && std::fabs(e[k]) > eps * (std::fabs(d[k]) + std::fabs(d[k + 1]))) ++k;
            if (k == l) break;
            if (sweep == 60) return false;
            // Wilkinson shift from the leading 2 x 2 block of rows l, l+1
            long double g = (d[l + 1] - d[l]) / (2.0L * e[l]);
            long double r = std::hypot(g, 1.0L);
            g = d[k] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            long double sn = 1.0L, cs = 1.0L, shift = 0.0L;
            bool deflated = false;
            for (int i = k - 1; i >= l; --i) {
                const long double f = sn * e[i], b = cs * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0L) {   // underflow: the block splits here
                    d[i + 1] -= shift;
                    e[k] = 0.0L;
                    deflated = true;
                    break;
                }
                sn = f / r;
                cs = g / r;
                g = d[i + 1] - shift;
                r = (d[i] - g) * sn + 2.0L * cs * b;
                shift = sn * r;
                d[i + 1] = g + shift;
                g = cs * r - b;
                for (int q = 0; q < m; ++q) {   // accumulate the rotation of columns i, i+1
                    long double &vi = V[size_t(q) * m + i], &vn = V[size_t(q) * m + i + 1];
                    const long double t = vn;
                    vn = sn * vi + cs * t;
                    vi = cs * vi - sn * t;
                }
            }
            if (deflated) continue;
            d[l] -= shift;
            e[l] = g;
            e[k] = 0.0L;
        }
    }
    return true;
}

// Eigenbases of the wall-bounded 3-point operators on a stretched axis:
// faces f[0..n] (strictly increasing), cell widths Delta_i = f[i+1] - f[i],
// centres c_i = (f[i] + f[i+1]) / 2, centre distances delta_i = c_i -
// c_{i-1}.  The operator L (flux form: the x rows of the staggered
// Laplacian over the local widths, with the same wall rows as the uniform
// kinds) is W^{-1} S with S symmetric and W the control widths (Delta_i for
// cell unknowns, delta_i for face unknowns), so it is diagonalised by the
// generalised eigenproblem S q = lambda W q.  Here through the symmetric
// T = W^{1/2} L W^{-1/2} = V Lambda V^T:
//   forward  xhat_a = sum_i F[i][a] x_i,  F = Wn^{1/2} V
//   inverse  x_i    = sum_a G[i][a] xhat_a, G = Wn^{-1/2} V
// with Wn = W / hbar (hbar = mean cell width), so that uniform faces give
// back the orthonormal bases above (F = G = Q) and a constant field of cell
// values maps onto mode 0 exactly as there: xhat_0 = sum_i Wn_i x_i /
// sqrt(n), and mode 0 inverts to the constant xhat_0 / sqrt(n).  Modes are
// ordered by increasing |lambda| (the pressure's mode 0 is its constant,
// lambda exactly 0), each with the sign that makes its largest component
// positive; XK_F keeps the wall slot as row and column 0 (zero, lambda 0).
// F and G are row-major n x n.  Returns false if the eigensolver fails.
static bool stretched_basis(int n, const std::vector<double> &f, int xk, std::vector<double> &F,
                            std::vector<double> &G, std::vector<double> &lam)
{
    F.assign(size_t(n) * n, 0.0);
    G.assign(size_t(n) * n, 0.0);
    lam.assign(n, 0.0);
    std::vector<long double> D(n), c(n), dl(n + 1, 0.0L);
    for (int i = 0; i < n; ++i) {
        D[i] = (long double)f[i + 1] - (long double)f[i];
        c[i] = 0.5L * ((long double)f[i] + (long double)f[i + 1]);
    }
    for (int i = 1; i < n; ++i) dl[i] = c[i] - c[i - 1];
    const long double hbar = ((long double)f[n] - (long double)f[0]) / n;
    const int first = (xk == XK_F) ? 1 : 0, m = n - first;   // unknowns first..n-1
    std::vector<long double> W(m), sd(m), so(m, 0.0L);      // S: diagonal, off-diagonal
    for (int r = 0; r < m; ++r) {
        const int i = r + first;
        if (xk == XK_F) {
            W[r] = dl[i];
            sd[r] = -(1.0L / D[i] + 1.0L / D[i - 1]);
            if (i + 1 <= n - 1) so[r] = 1.0L / D[i];
        } else {
            W[r] = D[i];
            long double diag = 0.0L;
            if (i + 1 < n) { diag -= 1.0L / dl[i + 1]; so[r] = 1.0L / dl[i + 1]; }
            if (i > 0) diag -= 1.0L / dl[i];
            if (xk == XK_C && i == 0) diag -= 2.0L / D[0];
            if (xk == XK_C && i == n - 1) diag -= 2.0L / D[n - 1];
            sd[r] = diag;
        }
    }
    std::vector<long double> td(m), te(m, 0.0L), V;
    for (int r = 0; r < m; ++r) {
        td[r] = sd[r] / W[r];
        if (r + 1 < m) te[r] = so[r] / std::sqrt(W[r] * W[r + 1]);
    }
    if (!tridiag_eigen(m, td, te, V)) return false;
    std::vector<int> ord(m);
    for (int a = 0; a < m; ++a) ord[a] = a;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return td[a] > td[b]; });
    long double wsum = 0.0L;
    for (int r = 0; r < m; ++r) wsum += W[r];
    for (int a = 0; a < m; ++a) {
        const int src = ord[a], col = a + first;
        // sign: the mode's largest component (the first of equal ones)
        // positive.  Not the first component: on a grid graded towards
        // both walls the high modes come in pairs localised at either wall,
        // degenerate to rounding, and a mode may vanish at the first wall.
        int rmax = 0;
        for (int r = 1; r < m; ++r)
            if (std::fabs(V[size_t(r) * m + src]) > std::fabs(V[size_t(rmax) * m + src])) rmax = r;
        const long double sg = V[size_t(rmax) * m + src] < 0 ? -1.0L : 1.0L;
        lam[col] = (double)td[src];
        for (int r = 0; r < m; ++r) {
            long double v = sg * V[size_t(r) * m + src];
            if (xk == XK_P && a == 0) v = std::sqrt(W[r] / wsum);   // the exact null vector
            const long double wn = std::sqrt(W[r] / hbar);
            F[size_t(r + first) * n + col] = (double)(wn * v);
            G[size_t(r + first) * n + col] = (double)(v / wn);
        }
    }
    if (xk == XK_P) lam[0] = 0.0;
    return true;
}

// Swizzle a K x N row-major matrix B into the per-lane fragment order of
// the 16x16x4 FP64 matrix-core instruction: for every 16-deep K chunk kc and
// 16-wide column block bj, lane l (0..63) holds four consecutive values
// B[16 kc + 4 (l/16) + t][16 bj + l%16], t = 0..3.
static void swizzle_b(const double *B, int K, int N, double *out)
{
    size_t o = 0;
    for (int kc = 0; kc < K / 16; ++kc)
        for (int bj = 0; bj < N / 16; ++bj)
            for (int l = 0; l < 64; ++l)
                for (int t = 0; t < 4; ++t)
                    out[o++] = B[size_t(16 * kc + 4 * (l / 16) + t) * N + 16 * bj + (l % 16)];
}
// Same for an M x K row-major A operand: lane l holds
// A[16 bi + l%16][16 kc + 4 (l/16) + t].
static void swizzle_a(const double *A, int M, int K, double *out)
{
    size_t o = 0;
    for (int kc = 0; kc < K / 16; ++kc)
        for (int bi = 0; bi < M / 16; ++bi)
            for (int l = 0; l < 64; ++l)
                for (int t = 0; t < 4; ++t)
                    out[o++] = A[size_t(16 * bi + (l % 16)) * K + 16 * kc + 4 * (l / 16) + t];
}

// The two H x H factors of the folded transform (H = N/2), from the basis
// Q[i][a] (grid index i, spectral index a; a < H cos and mean, a = H
// Nyquist, H + k sin mode k).  Row index i < H is the grid point paired
// with N - i; column index of s_* is k (k = 0 stands for the Nyquist mode).
//   c[i][a]     = Q[i][a]                         (a < H)
//   s_fwd[i][k] = Q[i][H+k] for i, k >= 1; s_fwd[0][0] = Q[H][H] (the O
//                 slot 0 carries X[H], whose only odd-side weight is the
//                 Nyquist one); other entries of row 0 / column 0 zero
//   s_inv[i][k] = Q[i][H+k] for k >= 1, 0 for k = 0 (the Nyquist input is
//                 even in i and is added outside the product)
struct FoldFactors {
    int h;
    std::vector<double> c, s_fwd, s_inv;
    FoldFactors(const std::vector<double> &Q, int N) : h(N / 2)
    {
        c.assign(size_t(h) * h, 0.0);
        s_fwd.assign(size_t(h) * h, 0.0);
        s_inv.assign(size_t(h) * h, 0.0);
        for (int i = 0; i < h; ++i)
            for (int a = 0; a < h; ++a) {
                c[size_t(i) * h + a] = Q[size_t(i) * N + a];
                if (a >= 1) {
                    s_inv[size_t(i) * h + a] = Q[size_t(i) * N + h + a];
                    if (i >= 1) s_fwd[size_t(i) * h + a] = Q[size_t(i) * N + h + a];
                }
            }
        s_fwd[0] = Q[size_t(h) * N + h];
    }
    std::vector<double> transposed(const std::vector<double> &m) const
    {
        std::vector<double> t(m.size());
        for (int i = 0; i < h; ++i)
            for (int j = 0; j < h; ++j) t[size_t(j) * h + i] = m[size_t(i) * h + j];
        return t;
    }
};

// bfloat16 bits of a float, rounded to nearest even (finite inputs).
static uint16_t bf16_rne(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
static double bf16_value(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return (double)f;
}
// Three-term bfloat16 split v = t0 + t1 + t2 (+ O(2^-24 |v|)); every
// remainder is formed exactly in double.
static void split3(double v, uint16_t t[3])
{
    double r = v;
    for (int q = 0; q < 3; ++q) {
        t[q] = bf16_rne((float)r);
        r -= bf16_value(t[q]);
    }
}
static std::vector<uint16_t> split_all(const double *M, size_t n)
{
    std::vector<uint16_t> out(3 * n);
    for (size_t i = 0; i < n; ++i) split3(M[i], &out[3 * i]);
    return out;
}
// Swizzle for the 16x16x32 bf16 matrix-core instruction, B operand (K x N):
// per 32-deep chunk kc and 16-wide column block bj, per split term t, lane l
// holds B[32 kc + 8 (l/16) + e][16 bj + l%16], e = 0..7 (16 bytes).
static void swizzle_b_split(const double *B, int K, int N, uint16_t *out)
{
    const std::vector<uint16_t> sp = split_all(B, size_t(K) * N);
    size_t o = 0;
    for (int kc = 0; kc < K / 32; ++kc)
        for (int bj = 0; bj < N / 16; ++bj)
            for (int t = 0; t < 3; ++t)
                for (int l = 0; l < 64; ++l)
                    for (int e = 0; e < 8; ++e)
                        out[o++] = sp[3 * (size_t(32 * kc + 8 * (l / 16) + e) * N + 16 * bj + (l % 16)) + t];
}
// A operand (M x K): lane l holds A[16 bi + l%16][32 kc + 8 (l/16) + e].
static void swizzle_a_split(const double *A, int M, int K, uint16_t *out)
{
    const std::vector<uint16_t> sp = split_all(A, size_t(M) * K);
    size_t o = 0;
    for (int kc = 0; kc < K / 32; ++kc)
        for (int bi = 0; bi < M / 16; ++bi)
            for (int t = 0; t < 3; ++t)
                for (int l = 0; l < 64; ++l)
                    for (int e = 0; e < 8; ++e)
                        out[o++] = sp[3 * (size_t(16 * bi + (l % 16)) * K + 32 * kc + 8 * (l / 16) + e) + t];
}

// The two H x H factors of a folded transform, split and swizzled chunk by
// chunk: per 32-deep chunk kc, factor f (0 cos, 1 sin), 16-block b, term t
// and lane l, the 8 values of that lane (B operand: F[32 kc + 8 (l/16) + e]
// [16 b + l%16]; A operand: F[16 b + l%16][32 kc + 8 (l/16) + e]).  One
// chunk of both factors is contiguous.
static void swizzle_split_pair(const std::vector<double> &F0, const std::vector<double> &F1, int H,
                               bool a_operand, uint16_t *out)
{
    const std::vector<uint16_t> s0 = split_all(F0.data(), F0.size());
    const std::vector<uint16_t> s1 = split_all(F1.data(), F1.size());
    size_t o = 0;
    for (int kc = 0; kc < H / 32; ++kc)
        for (int f = 0; f < 2; ++f) {
            const std::vector<uint16_t> &sp = f == 0 ? s0 : s1;
            for (int b = 0; b < H / 16; ++b)
                for (int t = 0; t < 3; ++t)
                    for (int l = 0; l < 64; ++l)
                        for (int e = 0; e < 8; ++e) {
                            const int k = 32 * kc + 8 * (l / 16) + e, m = 16 * b + (l % 16);
                            const size_t idx = a_operand ? size_t(m) * H + k : size_t(k) * H + m;
                            out[o++] = sp[3 * idx + t];
                        }
        }
}

// Everything a plan holds for one periodic axis depends only on its length
// n, its spacing h, which axis it is (x: B operand of the products, z: A
// operand) and whether the split tables are needed: the eigenbasis, the
// eigenvalues, and the blob images of the FP64 and split transforms along
// it.  Grids that share an axis (a serving mix whose y stretching differs
// from request to request) take these from a small process-wide cache.
struct AxisTables {
    std::vector<double> Q, lam;
    std::vector<double> Qi;            // stretched axis: the inverse basis G (else empty: G = Q)
    std::vector<double> f64[4];        // folded: fwd_c, fwd_s, inv_c, inv_s; plain: fwd, inv
    std::vector<uint16_t> split[2];    // fwd, inv (folded pairs or plain); empty without split
    size_t bytes() const
    {
        size_t b = (Q.size() + Qi.size() + lam.size()) * sizeof(double);
        for (const auto &v : f64) b += v.size() * sizeof(double);
        for (const auto &v : split) b += v.size() * sizeof(uint16_t);
        return b;
    }
};

// basis: -1 the periodic Fourier basis; XK_* a wall-bounded x basis (never
// folded: the folds rest on the Fourier basis's mirror symmetry), on the
// given faces when `faces` is not empty (stretched: forward F = Q and
// inverse G = Qi differ).  Returns null if the eigensolver fails.
static std::shared_ptr<const AxisTables> build_axis(int n, double h, bool z_axis, bool split, int basis,
                                                    const std::vector<double> &faces)
{
    auto t = std::make_shared<AxisTables>();
    if (basis < 0) fourier_basis(n, h, t->Q, t->lam);
    else if (faces.empty()) wall_basis(n, h, basis, t->Q, t->lam);
    else if (!stretched_basis(n, faces, basis, t->Q, t->Qi, t->lam)) return nullptr;
    const std::vector<double> &Q = t->Q;
    const std::vector<double> &Gi = t->Qi.empty() ? t->Q : t->Qi;   // inverse basis
    const int hn = n / 2;
    const size_t h2 = size_t(hn) * hn;
    const bool fourier = basis < 0;
    if (fourier && can_fold(n)) {
        FoldFactors f(Q, n);
        for (auto &v : t->f64) v.resize(h2);
        if (!z_axis) {
            swizzle_b(f.c.data(), hn, hn, t->f64[0].data());                   // forward: E Qc
            swizzle_b(f.s_fwd.data(), hn, hn, t->f64[1].data());               // forward: O Qs
            swizzle_b(f.transposed(f.c).data(), hn, hn, t->f64[2].data());     // inverse: Xc Qc^T
            swizzle_b(f.transposed(f.s_inv).data(), hn, hn, t->f64[3].data()); // inverse: Xs Qs^T
        } else {
            swizzle_a(f.transposed(f.c).data(), hn, hn, t->f64[0].data());     // forward: Qc^T E
            swizzle_a(f.transposed(f.s_fwd).data(), hn, hn, t->f64[1].data()); // forward: Qs^T O
            swizzle_a(f.c.data(), hn, hn, t->f64[2].data());                   // inverse: Qc Xc
            swizzle_a(f.s_inv.data(), hn, hn, t->f64[3].data());               // inverse: Qs Xs
        }
    } else {
        // tq = Q^T (forward, z), tg = G^T (inverse, x); G = Q unless stretched
        std::vector<double> tq(size_t(n) * n), tg(size_t(n) * n);
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < n; ++a) {
                tq[size_t(a) * n + i] = Q[size_t(i) * n + a];
                tg[size_t(a) * n + i] = Gi[size_t(i) * n + a];
            }
        t->f64[0].resize(size_t(n) * n);
        t->f64[1].resize(size_t(n) * n);
        if (!z_axis) {
            swizzle_b(Q.data(), n, n, t->f64[0].data());    // x forward: C = X Q
            swizzle_b(tg.data(), n, n, t->f64[1].data());   // x inverse: C = Xhat G^T
        } else {
            swizzle_a(tq.data(), n, n, t->f64[0].data());   // z forward: A = Q^T
            swizzle_a(Gi.data(), n, n, t->f64[1].data());   // z inverse: A = G
        }
    }
    if (split) {
        if (fourier && can_fold_split(n)) {
            FoldFactors f(Q, n);
            t->split[0].resize(size_t(3) * 2 * h2);
            t->split[1].resize(size_t(3) * 2 * h2);
            if (!z_axis) {
                swizzle_split_pair(f.c, f.s_fwd, hn, false, t->split[0].data());   // forward: E Qc, O Qs
                swizzle_split_pair(f.transposed(f.c), f.transposed(f.s_inv), hn, false, t->split[1].data());
            } else {
                swizzle_split_pair(f.transposed(f.c), f.transposed(f.s_fwd), hn, true, t->split[0].data());
                swizzle_split_pair(f.c, f.s_inv, hn, true, t->split[1].data());
            }
        } else {
            std::vector<double> tq(size_t(n) * n), tg(size_t(n) * n);
            for (int i = 0; i < n; ++i)
                for (int a = 0; a < n; ++a) {
                    tq[size_t(a) * n + i] = Q[size_t(i) * n + a];
                    tg[size_t(a) * n + i] = Gi[size_t(i) * n + a];
                }
            t->split[0].resize(size_t(3) * n * n);
            t->split[1].resize(size_t(3) * n * n);
            if (!z_axis) {
                swizzle_b_split(Q.data(), n, n, t->split[0].data());
                swizzle_b_split(tg.data(), n, n, t->split[1].data());
            } else {
                swizzle_a_split(tq.data(), n, n, t->split[0].data());
                swizzle_a_split(Gi.data(), n, n, t->split[1].data());
            }
        }
    }
    return t;
}

void plain_transform_table(const Plan &p, bool z_axis, int kind, bool inverse, std::vector<double> &out)
{
    const int n = z_axis ? p.nz : p.nx;
    const std::vector<double> &Q = z_axis ? p.qz[kind] : p.qx[kind];
    const std::vector<double> &G = z_axis ? p.gz[kind] : p.gx[kind];
    out.assign(size_t(n) * n, 0.0);
    std::vector<double> t(size_t(n) * n);
    const std::vector<double> &M = inverse ? G : Q;
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < n; ++a) t[size_t(a) * n + i] = M[size_t(i) * n + a];
    if (!z_axis) swizzle_b(inverse ? t.data() : Q.data(), n, n, out.data());   // X Q, Xhat G^T
    else swizzle_a(inverse ? G.data() : t.data(), n, n, out.data());           // Q^T X, G Xhat
}

// Cache of axis tables, at most AXIS_CACHE_BYTES of host memory (oldest
// entries dropped first).  Plans copy what they need, so dropping an entry
// never affects an existing plan.
constexpr size_t AXIS_CACHE_BYTES = size_t(256) << 20;
static std::shared_ptr<const AxisTables> axis_tables(int n, double h, bool z_axis, bool split,
                                                     int basis = -1,
                                                     const std::vector<double> &faces = {})
{
    struct Entry {
        int n;
        double h;
        bool z, split;
        int basis;
        std::vector<double> faces;
        std::shared_ptr<const AxisTables> t;
    };
    static std::mutex mu;
    static std::vector<Entry> cache;
    {
        std::lock_guard<std::mutex> lock(mu);
        for (const Entry &e : cache)
            if (e.n == n && e.h == h && e.z == z_axis && e.split == split && e.basis == basis &&
                e.faces == faces)
                return e.t;
    }
    std::shared_ptr<const AxisTables> t = build_axis(n, h, z_axis, split, basis, faces);
    if (!t) return t;
    std::lock_guard<std::mutex> lock(mu);
    size_t total = t->bytes();
    for (const Entry &e : cache) total += e.t->bytes();
    while (!cache.empty() && total > AXIS_CACHE_BYTES) {
        total -= cache.front().t->bytes();
        cache.erase(cache.begin());
    }
    if (t->bytes() <= AXIS_CACHE_BYTES) cache.push_back(Entry{n, h, z_axis, split, basis, faces, t});
    return t;
}

// The per-index geometry of a stretched wall-bounded axis on faces f[0..n]
// (StretchSlot layout): SG_SLOTS arrays of n doubles, from long-double
// widths.
static std::vector<double> stretch_geometry(const std::vector<double> &f)
{
    const int n = (int)f.size() - 1;
    std::vector<long double> D(n), dl(n + 1, 0.0L);
    for (int i = 0; i < n; ++i) D[i] = (long double)f[i + 1] - (long double)f[i];
    for (int i = 1; i < n; ++i) dl[i] = 0.5L * (D[i - 1] + D[i]);
    const long double hbar = ((long double)f[n] - (long double)f[0]) / n;
    std::vector<double> g(size_t(SG_SLOTS) * n, 0.0);
    auto at = [&](int slot, int i) -> double & { return g[size_t(slot) * n + i]; };
    for (int i = 0; i < n; ++i) {
        at(SG_RC, i) = (double)(1.0L / D[i]);
        at(SG_RF, i) = i > 0 ? (double)(1.0L / dl[i]) : 0.0;
        at(SG_WN, i) = (double)(D[i] / hbar);
        const long double e = i + 1 < n ? 1.0L / (dl[i + 1] * D[i]) : 0.0L;
        const long double w = i > 0 ? 1.0L / (dl[i] * D[i]) : 0.0L;
        at(sg_ae(XK_P), i) = (double)e;
        at(sg_aw(XK_P), i) = (double)w;
        at(sg_ae(XK_C), i) = (double)(i + 1 < n ? e : 1.0L / (D[i] * D[i]));
        at(sg_aw(XK_C), i) = (double)(i > 0 ? w : 1.0L / (D[i] * D[i]));
        at(sg_ae(XK_F), i) = i > 0 ? (double)(1.0L / (D[i] * dl[i])) : 0.0;
        at(sg_aw(XK_F), i) = i > 0 ? (double)(1.0L / (D[i - 1] * dl[i])) : 0.0;
    }
    return g;
}

ibs_status build_plan(const ibs_grid_desc &d, Plan *&out)
{
    if (d.nx < 16 || d.nz < 16 || d.nx > 1024 || d.nz > 1024 || d.nx % 16 || d.nz % 16) {
        set_error("nx and nz must be multiples of 16 in [16, 1024]");
        return IBS_ERR_UNSUPPORTED;
    }
    if (d.ny < 2 || d.ny > 768) {   // the tridiagonal shapes cover up to 800 system rows
        set_error("ny must be in [2, 768]");
        return IBS_ERR_UNSUPPORTED;
    }
    const bool walls_y = d.bc_y_vel == IBS_DIRICHLET && d.bc_y_p == IBS_NEUMANN;
    const bool periodic_y = d.bc_y_vel == IBS_PERIODIC && d.bc_y_p == IBS_PERIODIC;
    if ((d.bc_x != IBS_PERIODIC && d.bc_x != IBS_DIRICHLET) ||
        (d.bc_z != IBS_PERIODIC && d.bc_z != IBS_DIRICHLET) || !(walls_y || periodic_y)) {
        set_error("supported: x and z each periodic or walls (IBS_DIRICHLET: Dirichlet velocity, "
                  "Neumann pressure), and in y either Dirichlet velocity / Neumann pressure walls "
                  "or periodic (triply periodic)");
        return IBS_ERR_UNSUPPORTED;
    }
    if (periodic_y && !cyclic_rows_supported(d.ny)) {
        set_error("periodic y needs ny in {48, 64, 80, 96, 128, 160, 192, 256, 320, 384, 512}");
        return IBS_ERR_UNSUPPORTED;
    }
    if (d.precision < IBS_FP64 || d.precision > IBS_REFINED_AUTO) {
        set_error("unknown precision");
        return IBS_ERR_INVALID_ARG;
    }
    if (d.precision == IBS_REFINED_FP16X2 || d.precision == IBS_REFINED_AUTO) {
        set_error("only the bfloat16x3 split scheme is built (IBS_REFINED_BF16X3); "
                  "IBS_REFINED_FP16X2 and IBS_REFINED_AUTO are not served");
        return IBS_ERR_UNSUPPORTED;
    }
    if (d.max_iter < 0 || d.max_iter > MAX_PASSES) {
        set_error("max_iter must be in [0, " + std::to_string(MAX_PASSES) + "]");
        return IBS_ERR_INVALID_ARG;
    }
    if (!(d.tol >= 0.0) && !(d.tol <= 0.0)) {
        set_error("tol must not be NaN");
        return IBS_ERR_INVALID_ARG;
    }
    if (d.precision != IBS_FP64 && (d.nx % 32 || d.nz % 32 || d.nx > 512 || d.nz > 512)) {
        set_error("the refined path needs nx and nz to be multiples of 32, at most 512");
        return IBS_ERR_UNSUPPORTED;
    }
    if (!(std::isfinite(d.beta)) || d.beta < 0.0 || d.beta > 10.0) {
        set_error("beta must be in [0, 10]");
        return IBS_ERR_INVALID_ARG;
    }
    if ((d.x_faces && d.bc_x != IBS_DIRICHLET) || (d.z_faces && d.bc_z != IBS_DIRICHLET)) {
        set_error("x_faces / z_faces (a stretched x or z) need walls along that axis (IBS_DIRICHLET)");
        return IBS_ERR_UNSUPPORTED;
    }
    // faces of a stretched x or z: finite and strictly increasing
    auto faces_ok = [](const double *f, int n) {
        for (int i = 0; i <= n; ++i)
            if (!std::isfinite(f[i]) || (i > 0 && !(f[i] - f[i - 1] > 0.0))) return false;
        return true;
    };
    if ((d.x_faces && !faces_ok(d.x_faces, d.nx)) || (d.z_faces && !faces_ok(d.z_faces, d.nz))) {
        set_error("x_faces / z_faces must be finite and strictly increasing");
        return IBS_ERR_INVALID_ARG;
    }
    Plan *p = new (std::nothrow) Plan();
    if (!p) { set_error("out of host memory"); return IBS_ERR_INVALID_ARG; }
    p->desc = d;
    p->desc.y_faces = nullptr;
    p->desc.x_faces = nullptr;
    p->desc.z_faces = nullptr;
    p->py = periodic_y;
    p->wx = d.bc_x == IBS_DIRICHLET;
    p->wz = d.bc_z == IBS_DIRICHLET;
    p->sx = d.x_faces != nullptr;
    p->sz = d.z_faces != nullptr;
    double lx = d.lx > 0 ? d.lx : 1.0, lz = d.lz > 0 ? d.lz : 1.0;
    const double ly = d.ly > 0 ? d.ly : 1.0;
    if (p->sx) lx = d.x_faces[d.nx] - d.x_faces[0];
    if (p->sz) lz = d.z_faces[d.nz] - d.z_faces[0];
    p->desc.lx = lx; p->desc.ly = ly; p->desc.lz = lz;
    if (p->desc.tol <= 0) p->desc.tol = 1e-10;
    const int nx = d.nx, ny = d.ny, nz = d.nz;
    p->nx = nx; p->ny = ny; p->nz = nz;
    p->hx = lx / nx;   // the mean width on a stretched axis
    p->hz = lz / nz;
    p->xf.resize(nx + 1);
    p->zf.resize(nz + 1);
    for (int i = 0; i <= nx; ++i) p->xf[i] = p->sx ? d.x_faces[i] : p->hx * i;
    for (int k = 0; k <= nz; ++k) p->zf[k] = p->sz ? d.z_faces[k] : p->hz * k;

    // y grid: tanh-stretched faces (uniform for beta = 0), centres midway
    p->yf.resize(ny + 1);
    for (int j = 0; j <= ny; ++j) {
        if (d.y_faces) {
            p->yf[j] = d.y_faces[j];
        } else if (d.beta == 0.0) {
            p->yf[j] = ly * (double)j / (double)ny;
        } else {
            double t = std::tanh(d.beta * (2.0 * (double)j / (double)ny - 1.0));
            p->yf[j] = 0.5 * ly * (1.0 + t / std::tanh(d.beta));
        }
    }
    p->yc.resize(ny);
    p->dyc.resize(ny);
    p->dyf.assign(ny + 1, 0.0);
    for (int j = 0; j < ny; ++j) {
        p->yc[j] = 0.5 * (p->yf[j] + p->yf[j + 1]);
        p->dyc[j] = p->yf[j + 1] - p->yf[j];
        if (!(p->dyc[j] > 0.0) || !std::isfinite(p->dyc[j])) {
            set_error("y faces must be finite and strictly increasing");
            delete p;
            return IBS_ERR_INVALID_ARG;
        }
    }
    for (int j = 1; j < ny; ++j) p->dyf[j] = p->yc[j] - p->yc[j - 1];
    // conditioning: no cell below MIN_CELL_FRACTION of its axis's length
    {
        auto min_fraction = [](const std::vector<double> &f) {
            double m = f[1] - f[0];
            for (size_t i = 1; i + 1 < f.size(); ++i) m = std::min(m, f[i + 1] - f[i]);
            return m / (f.back() - f.front());
        };
        if (min_fraction(p->yf) < MIN_CELL_FRACTION || min_fraction(p->xf) < MIN_CELL_FRACTION ||
            min_fraction(p->zf) < MIN_CELL_FRACTION) {
            set_error("a cell narrower than 1e-7 of its axis's length (the stretching is too strong): "
                      "the operators' condition number exceeds what FP64 residuals resolve");
            delete p;
            return IBS_ERR_UNSUPPORTED;
        }
    }
    // periodic y: the centres of cells ny-1 and 0 are (Delta_{ny-1} +
    // Delta_0)/2 apart across the wrap; that distance is delta_0 = delta_ny
    if (p->py) p->dyf[0] = p->dyf[ny] = 0.5 * (p->dyc[0] + p->dyc[ny - 1]);

    // y operators, one tridiagonal row per unknown (unweighted Laplacian in y)
    p->rows[KIND_P] = ny;
    p->rows[KIND_C] = ny;
    p->rows[KIND_F] = ny + 1;
    p->rows[KIND_PF] = ny;
    for (int kd = 0; kd < NUM_KINDS; ++kd) {
        p->lo[kd].assign(ny + 1, 0.0);
        p->di[kd].assign(ny + 1, 0.0);
        p->up[kd].assign(ny + 1, 0.0);
    }
    for (int j = 0; p->py && j < ny; ++j) {
        // periodic y: the interior rows everywhere; lo[0] couples row 0 to
        // row ny-1 and up[ny-1] row ny-1 to row 0 (the cyclic corners).
        // Cells (p, u, w): (F_{j+1/2} - F_{j-1/2}) / Delta_j, fluxes over
        // delta; faces (v): fluxes over Delta, divided by delta_j.
        const double lo = 1.0 / (p->dyf[j] * p->dyc[j]);
        const double up = 1.0 / (p->dyf[j + 1] * p->dyc[j]);
        for (int kd : {KIND_P, KIND_C}) {
            p->lo[kd][j] = lo;
            p->up[kd][j] = up;
            p->di[kd][j] = -(lo + up);
        }
        const double flo = 1.0 / (p->dyf[j] * p->dyc[(j + ny - 1) % ny]);
        const double fup = 1.0 / (p->dyf[j] * p->dyc[j]);
        p->lo[KIND_PF][j] = flo;
        p->up[KIND_PF][j] = fup;
        p->di[KIND_PF][j] = -(flo + fup);
    }
    for (int j = 0; !p->py && j < ny; ++j) {
        // cell-centre rows: (F_{j+1/2} - F_{j-1/2}) / Delta_j
        double lo = (j > 0) ? 1.0 / (p->dyf[j] * p->dyc[j]) : 0.0;
        double up = (j + 1 < ny) ? 1.0 / (p->dyf[j + 1] * p->dyc[j]) : 0.0;
        p->lo[KIND_P][j] = lo;
        p->up[KIND_P][j] = up;
        p->di[KIND_P][j] = -(lo + up);  // Neumann: no wall flux
        double wall = 0.0;              // Dirichlet: mirror ghost, flux 2 f / Delta
        if (j == 0) wall += 2.0 / (p->dyc[0] * p->dyc[0]);
        if (j == ny - 1) wall += 2.0 / (p->dyc[ny - 1] * p->dyc[ny - 1]);
        p->lo[KIND_C][j] = lo;
        p->up[KIND_C][j] = up;
        p->di[KIND_C][j] = -(lo + up) - wall;
    }
    for (int j = 1; !p->py && j < ny; ++j) {
        // face rows: ((v_{j+1}-v_j)/Delta_j - (v_j-v_{j-1})/Delta_{j-1}) / delta_j;
        // the wall rows 0 and ny stay zero (their unknowns are pinned to 0)
        double lo = 1.0 / (p->dyf[j] * p->dyc[j - 1]);
        double up = 1.0 / (p->dyf[j] * p->dyc[j]);
        p->lo[KIND_F][j] = lo;
        p->up[KIND_F][j] = up;
        p->di[KIND_F][j] = -(lo + up);
    }

    const bool split = d.precision != IBS_FP64;
    // x: one Fourier table set (periodic), or one per x kind (walls)
    const std::vector<double> no_faces;
    std::shared_ptr<const AxisTables> ax[NUM_XK];
    for (int k = 0; k < NUM_XK; ++k)
        ax[k] = (p->wx || k == 0) ? axis_tables(nx, p->hx, false, split, p->wx ? k : -1,
                                                p->sx ? p->xf : no_faces)
                                  : ax[0];
    std::shared_ptr<const AxisTables> az[NUM_XK];
    for (int k = 0; k < NUM_XK; ++k)
        az[k] = (p->wz || k == 0) ? axis_tables(nz, p->hz, true, split, p->wz ? k : -1,
                                                p->sz ? p->zf : no_faces)
                                  : az[0];
    for (int k = 0; k < NUM_XK; ++k)
        if (!ax[k] || !az[k]) {
            set_error("the eigensolver of a stretched axis did not converge");
            delete p;
            return IBS_ERR_INVALID_ARG;
        }
    for (int k = 0; k < NUM_XK; ++k) {
        p->qx[k] = ax[k]->Q;
        p->gx[k] = ax[k]->Qi.empty() ? ax[k]->Q : ax[k]->Qi;
        p->lam_x[k] = ax[k]->lam;
        p->qz[k] = az[k]->Q;
        p->gz[k] = az[k]->Qi.empty() ? az[k]->Q : az[k]->Qi;
        p->lam_z[k] = az[k]->lam;
    }
    const int nxk = p->wx ? NUM_XK : 1;   // distinct x tables
    const int nzk = p->wz ? NUM_XK : 1;   // distinct z tables

    // blob layout
    BlobLayout &L = p->lay;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
    const bool fold_x = x_folds(*p), fold_z = z_folds(*p);
    const size_t hx2 = size_t(nx / 2) * (nx / 2), hz2 = size_t(nz / 2) * (nz / 2);
    for (int k = 0; k < NUM_XK; ++k) {
        L.bx_fwd[k] = k < nxk ? take(fold_x ? 0 : sizeof(double) * nx * nx) : L.bx_fwd[0];
        L.bx_inv[k] = k < nxk ? take(fold_x ? 0 : sizeof(double) * nx * nx) : L.bx_inv[0];
    }
    for (int k = 0; k < NUM_XK; ++k) {
        L.az_fwd[k] = k < nzk ? take(fold_z ? 0 : sizeof(double) * nz * nz) : L.az_fwd[0];
        L.az_inv[k] = k < nzk ? take(fold_z ? 0 : sizeof(double) * nz * nz) : L.az_inv[0];
    }
    L.fx_fwd_c = take(fold_x ? sizeof(double) * hx2 : 0);
    L.fx_fwd_s = take(fold_x ? sizeof(double) * hx2 : 0);
    L.fx_inv_c = take(fold_x ? sizeof(double) * hx2 : 0);
    L.fx_inv_s = take(fold_x ? sizeof(double) * hx2 : 0);
    L.fz_fwd_c = take(fold_z ? sizeof(double) * hz2 : 0);
    L.fz_fwd_s = take(fold_z ? sizeof(double) * hz2 : 0);
    L.fz_inv_c = take(fold_z ? sizeof(double) * hz2 : 0);
    L.fz_inv_s = take(fold_z ? sizeof(double) * hz2 : 0);
    for (int k = 0; k < NUM_XK; ++k) L.lam_x[k] = k < nxk ? take(sizeof(double) * nx) : L.lam_x[0];
    for (int k = 0; k < NUM_XK; ++k) L.lam_z[k] = k < nzk ? take(sizeof(double) * nz) : L.lam_z[0];
    for (int kd = 0; kd < NUM_KINDS; ++kd) {
        L.lo[kd] = take(sizeof(double) * (ny + 1));
        L.di[kd] = take(sizeof(double) * (ny + 1));
        L.up[kd] = take(sizeof(double) * (ny + 1));
    }
    L.wy = take(sizeof(double) * ny);
    L.dyc = take(sizeof(double) * ny);
    L.dyf = take(sizeof(double) * (ny + 1));
    const bool sfold_x = split && x_folds_split(*p), sfold_z = split && z_folds_split(*p);
    for (int k = 0; k < NUM_XK; ++k) {
        L.sx_fwd[k] = k < nxk ? take(split && !sfold_x ? sizeof(uint16_t) * 3 * nx * nx : 0) : L.sx_fwd[0];
        L.sx_inv[k] = k < nxk ? take(split && !sfold_x ? sizeof(uint16_t) * 3 * nx * nx : 0) : L.sx_inv[0];
    }
    for (int k = 0; k < NUM_XK; ++k) {
        L.sz_fwd[k] = k < nzk ? take(split && !sfold_z ? sizeof(uint16_t) * 3 * nz * nz : 0) : L.sz_fwd[0];
        L.sz_inv[k] = k < nzk ? take(split && !sfold_z ? sizeof(uint16_t) * 3 * nz * nz : 0) : L.sz_inv[0];
    }
    L.sxf_fwd = take(sfold_x ? sizeof(uint16_t) * 3 * 2 * hx2 : 0);
    L.sxf_inv = take(sfold_x ? sizeof(uint16_t) * 3 * 2 * hx2 : 0);
    L.szf_fwd = take(sfold_z ? sizeof(uint16_t) * 3 * 2 * hz2 : 0);
    L.szf_inv = take(sfold_z ? sizeof(uint16_t) * 3 * 2 * hz2 : 0);
    // FP64 lane of the refined pressure pencils: a 32-wide x-tile of z-mode
    // c joins it when any of its pencils is singular or has a condition
    // bound 1 + g/|s| above LANE64_KAPPA (LANE64_KAPPA_CYCLIC when y is periodic)
    std::vector<uint32_t> lane_mask;
    std::vector<int> lane_list;
    if (split) {
        double g = 0.0;
        for (int j = 0; j < ny; ++j)
            g = std::max(g, std::fabs(p->lo[KIND_P][j]) + std::fabs(p->di[KIND_P][j]) + std::fabs(p->up[KIND_P][j]));
        lane_mask.assign(nz, 0u);
        for (int c = 0; c < nz; ++c)
            for (int t = 0; t < nx / 32; ++t) {
                bool need = false;
                for (int a = 32 * t; a < 32 * t + 32 && !need; ++a) {
                    const double sabs = std::fabs(p->lam_x[XK_P][a] + p->lam_z[XK_P][c]);
                    need = sabs == 0.0 || 1.0 + g / sabs > (p->py ? LANE64_KAPPA_CYCLIC : LANE64_KAPPA);
                }
                if (need) {
                    lane_mask[c] |= 1u << t;
                    lane_list.push_back((c << 8) | t);
                }
            }
    }
    p->lane_len = (int)lane_list.size();
    L.lane_mask = take(sizeof(uint32_t) * lane_mask.size());
    L.lane_list = take(sizeof(int) * lane_list.size());
    L.sgx = take(p->sx ? sizeof(double) * SG_SLOTS * nx : 0);
    L.sgz = take(p->sz ? sizeof(double) * SG_SLOTS * nz : 0);
    L.total = o;
    p->blob.assign(L.total, 0);
    auto put = [&](size_t off, const double *src, size_t n) {
        std::memcpy(p->blob.data() + off, src, n * sizeof(double));
    };
    auto put16 = [&](size_t off, const std::vector<uint16_t> &src) {
        std::memcpy(p->blob.data() + off, src.data(), src.size() * sizeof(uint16_t));
    };
    if (fold_x) {
        put(L.fx_fwd_c, ax[0]->f64[0].data(), hx2);
        put(L.fx_fwd_s, ax[0]->f64[1].data(), hx2);
        put(L.fx_inv_c, ax[0]->f64[2].data(), hx2);
        put(L.fx_inv_s, ax[0]->f64[3].data(), hx2);
    } else {
        for (int k = 0; k < nxk; ++k) {
            put(L.bx_fwd[k], ax[k]->f64[0].data(), size_t(nx) * nx);
            put(L.bx_inv[k], ax[k]->f64[1].data(), size_t(nx) * nx);
        }
    }
    if (fold_z) {
        put(L.fz_fwd_c, az[0]->f64[0].data(), hz2);
        put(L.fz_fwd_s, az[0]->f64[1].data(), hz2);
        put(L.fz_inv_c, az[0]->f64[2].data(), hz2);
        put(L.fz_inv_s, az[0]->f64[3].data(), hz2);
    } else {
        for (int k = 0; k < nzk; ++k) {
            put(L.az_fwd[k], az[k]->f64[0].data(), size_t(nz) * nz);
            put(L.az_inv[k], az[k]->f64[1].data(), size_t(nz) * nz);
        }
    }
    if (split) {
        if (sfold_x) {
            put16(L.sxf_fwd, ax[0]->split[0]);
            put16(L.sxf_inv, ax[0]->split[1]);
        } else {
            for (int k = 0; k < nxk; ++k) {
                put16(L.sx_fwd[k], ax[k]->split[0]);
                put16(L.sx_inv[k], ax[k]->split[1]);
            }
        }
        if (sfold_z) {
            put16(L.szf_fwd, az[0]->split[0]);
            put16(L.szf_inv, az[0]->split[1]);
        } else {
            for (int k = 0; k < nzk; ++k) {
                put16(L.sz_fwd[k], az[k]->split[0]);
                put16(L.sz_inv[k], az[k]->split[1]);
            }
        }
    }
    if (!lane_mask.empty()) std::memcpy(p->blob.data() + L.lane_mask, lane_mask.data(), 4 * lane_mask.size());
    if (!lane_list.empty()) std::memcpy(p->blob.data() + L.lane_list, lane_list.data(), 4 * lane_list.size());
    for (int k = 0; k < nxk; ++k) put(L.lam_x[k], p->lam_x[k].data(), nx);
    for (int k = 0; k < nzk; ++k) put(L.lam_z[k], p->lam_z[k].data(), nz);
    for (int kd = 0; kd < NUM_KINDS; ++kd) {
        put(L.lo[kd], p->lo[kd].data(), ny + 1);
        put(L.di[kd], p->di[kd].data(), ny + 1);
        put(L.up[kd], p->up[kd].data(), ny + 1);
    }
    put(L.wy, p->dyc.data(), ny);
    put(L.dyc, p->dyc.data(), ny);
    put(L.dyf, p->dyf.data(), ny + 1);
    if (p->sx) {
        const std::vector<double> g = stretch_geometry(p->xf);
        put(L.sgx, g.data(), g.size());
    }
    if (p->sz) {
        const std::vector<double> g = stretch_geometry(p->zf);
        put(L.sgz, g.data(), g.size());
    }
    out = p;
    return IBS_OK;
}

}  // namespace ibs
