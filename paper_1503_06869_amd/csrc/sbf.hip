// sbf.hip -- the slender-body formulation (Sec. 3 of the paper) on gfx950:
// moments of the free-space Green's function between every pair of fibers
// (Eq. Gnonper, integrals of the form of Eq. theta_def), the dense Legendre
// system of Eqs. sev_fils and extra_cond with the expansion of Eq.
// force_exp, solved by restarted GMRES, the velocities of Eqs. xadot and
// padot, and Adams-Bashforth-2 time stepping.  C ABI in include/sbf.h.
//
// Layout.  The moments form one dense symmetric FP64 matrix W of order
// D = 3 M (N + 1): row (m, n, a), column (m', k, b) holds
//   Theta^{n,k}_{mm'}[a][b] = int int G(R(s, s'))_ab P_k(s'/l) P_n(s/l) ds' ds,
//   R = x_m + s p_m - x_m' - s' p_m',
// n, k = 0..N, zero for m = m' (a fiber does not see itself through G).
// Every vector (Krylov basis, solution, right-hand side) uses the same
// (m, k, b) layout, its k = 0 entries zero except where the known force
// part F/(2l) is put in.  Then every product with W is one GEMV, the
// system operator is that GEMV followed by 3x3 block operations per (m, n),
// and the velocities come from the n = 0 and n = 1 rows of W [F/(2l); a].
//
// G(R) and G(-R) are equal and symmetric, so Theta^{k,n}_{m'm} is the
// transpose of Theta^{n,k}_{mm'} and W = W^T.  Only its upper triangle is
// stored, as 64 x 64 tiles (i, j), i <= j, packed row after row, each tile
// row-major; the diagonal tiles are stored whole, padding rows and columns
// beyond D are zero.  A product y = W x reads every stored tile once and
// uses it twice, W_ij x_j for the rows of block i and W_ij^T x_i for the
// rows of block j (i < j), writing each into its own slot of a partial-sum
// array part[slot][row] (row sums per chunk of tiles of a tile row, column
// sums per tile); a second pass adds the slots of each row in a fixed order.
//
// Bound: the moments are FP64 ALU work (M^2/2 pairs x (3 nq)^2 Green's
// function evaluations, each pair giving both of its blocks of W); each
// GMRES iteration streams the stored half of W once (about D^2/2 x 8
// bytes, HBM bound).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/sbf.h"

namespace sbfk {

constexpr int MAXN = 8;        // Legendre modes supported (N <= 8)
constexpr int MAXR = 64;       // Krylov dimension
constexpr int TS = 64;         // tile edge of the packed moment matrix

struct Consts {
    int M, N, Q, D;            // fibers, modes, quadrature points per fiber, order of W
    int nt;                    // tiles per side, ceil(D / TS)
    double l, L, r, d, mu;
};

// first element of tile (i, j), i <= j, in the packed upper triangle
__host__ __device__ __forceinline__ size_t tile_base(int i, int j, int nt)
{
    // rows r < i hold nt - r tiles each: i nt - i (i - 1)/2 = i (2 nt - i + 1)/2
    return (size_t(i) * (2 * size_t(nt) - size_t(i) + 1) / 2 + size_t(j - i)) * (TS * TS);
}

// packed tiles of the upper triangle for nt tiles per side
__host__ __device__ __forceinline__ size_t packed_tiles(int nt) { return size_t(nt) * size_t(nt + 1) / 2; }

// ------------------------------------------------------------------ moments
// 1/sqrt(x) for x > 0: the hardware estimate refined by two Newton steps
// y <- y + y (1 - x y^2)/2 (each at least doubles the correct bits).
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

// entry (R, C), R < C, of the symmetric matrix into the packed upper
// triangle (a diagonal tile is stored whole: its mirror entry too)
__device__ __forceinline__ void put_sym(double *W, int nt, int R, int C, double v)
{
    const int bi = R / TS, bj = C / TS, ri = R % TS, ci = C % TS;
    double *t = W + tile_base(bi, bj, nt);
    t[ri * TS + ci] = v;
    if (bi == bj) t[ci * TS + ri] = v;
}

// Sums over the inner points s'_j for the outer point s_i of the pair:
// acc[k] = sum_j w_j P_k(s_j) (alpha, beta R R^T entries) of G(R_ij).
template <int NP1>
__device__ __forceinline__ void moment_point(int i, const double (&xm)[3], const double (&pm)[3],
                                             const double (&xn)[3], const double (&pn)[3], double h,
                                             const Consts &c, const double *__restrict__ sq,
                                             const double *__restrict__ wl, double (&acc)[NP1][7])
{
#pragma unroll
    for (int k = 0; k < NP1; ++k)
#pragma unroll
        for (int e = 0; e < 7; ++e) acc[k][e] = 0.0;
    const double si = sq[i];
    const double b0 = xm[0] + si * pm[0] - xn[0], b1 = xm[1] + si * pm[1] - xn[1], b2 = xm[2] + si * pm[2] - xn[2];
    for (int j = 0; j < c.Q; ++j) {
        const double sj = sq[j];
        const double R0 = b0 - sj * pn[0], R1 = b1 - sj * pn[1], R2 = b2 - sj * pn[2];
        const double r2 = R0 * R0 + R1 * R1 + R2 * R2;
        const double inv = rsqrt_nr(r2);
        const double inv2 = inv * inv, inv3 = inv * inv2;
        const double alpha = inv + h * inv3;
        const double beta = inv3 - 3.0 * h * inv3 * inv2;
        const double g[7] = {alpha, beta * R0 * R0, beta * R0 * R1, beta * R0 * R2,
                             beta * R1 * R1, beta * R1 * R2, beta * R2 * R2};
#pragma unroll
        for (int k = 0; k < NP1; ++k) {
            const double wk = wl[k * c.Q + j];
#pragma unroll
            for (int e = 0; e < 7; ++e) acc[k][e] += wk * g[e];
        }
    }
}

// Moments for Q <= 64: workgroup b takes the pairs b PB .. b PB + PB - 1
// of the list of pairs m < m' (row by row; the pair gives both blocks of W,
// the diagonal blocks stay at the zero the packed matrix was cleared to).
// Thread t serves pair slot t / Q and its outer quadrature point
// s_i, i = t % Q: it sums over the inner points s'_j, per trial mode k, the
// scalar part alpha and the six components of beta R R^T of
// G = alpha I + beta R R^T (moment_point); the outer sums with P_n(s_i)
// follow one trial mode k at a time through LDS ([Q][7] per pair, then
// out[NP1][NP1][7] per pair).  wl[k][j] = w_j P_k(s_j).
__device__ __forceinline__ void pair_of(long long p, int M, int &m, int &mp)
{
    // start(m) = m (2M - m - 1)/2 pairs precede row m
    const double b = 2.0 * M - 1.0;
    long long r = (long long)((b - sqrt(b * b - 8.0 * double(p))) * 0.5);
    r = r < 0 ? 0 : (r > M - 2 ? M - 2 : r);
    while (r > 0 && r * (2LL * M - r - 1) / 2 > p) --r;
    while (r + 1 <= M - 2 && (r + 1) * (2LL * M - r - 2) / 2 <= p) ++r;
    m = int(r);
    mp = int(r + 1 + (p - r * (2LL * M - r - 1) / 2));
}

// symmetric 3x3 index of (a, b) into the six beta components
__device__ __forceinline__ int sym_index(int a, int b) { return a == b ? (a == 0 ? 1 : (a == 1 ? 4 : 6)) : (a + b == 1 ? 2 : (a + b == 2 ? 3 : 5)); }

template <int NP1>
__global__ __launch_bounds__(256) void k_theta(const double *__restrict__ X, const double *__restrict__ p, Consts c,
                                               const double *__restrict__ sq, const double *__restrict__ wl,
                                               double *__restrict__ W, int PB, long long P)
{
    // LDS: wl [NP1][Q]; the pairs' (m, m') [PB][2]; per pair [Q][7] then out[NP1][NP1][7]
    extern __shared__ double sh[];
    const int st = 3 * NP1, per = c.Q * 7 + NP1 * NP1 * 7;
    double *swl = sh;
    int *pairs = reinterpret_cast<int *>(sh + NP1 * c.Q);
    double *pd = sh + NP1 * c.Q + (PB + 1) / 2 * 2;
    const int t = int(threadIdx.x), slot = t / c.Q, i = t % c.Q;
    const long long p0 = (long long)blockIdx.x * PB;
    const bool act = slot < PB && p0 + slot < P;
    for (int e = t; e < NP1 * c.Q; e += int(blockDim.x)) swl[e] = wl[e];
    int m = 0, mp = 0;
    if (act) {
        pair_of(p0 + slot, c.M, m, mp);
        if (i == 0) {
            pairs[2 * slot] = m;
            pairs[2 * slot + 1] = mp;
        }
    }
    double acc[NP1][7];
    if (act) {
        const double xm[3] = {X[3 * m], X[3 * m + 1], X[3 * m + 2]};
        const double pm[3] = {p[3 * m], p[3 * m + 1], p[3 * m + 2]};
        const double xn[3] = {X[3 * mp], X[3 * mp + 1], X[3 * mp + 2]};
        const double pn[3] = {p[3 * mp], p[3 * mp + 1], p[3 * mp + 2]};
        moment_point<NP1>(i, xm, pm, xn, pn, 0.5 * c.r * c.r, c, sq, wl, acc);
    }
#pragma unroll
    for (int k = 0; k < NP1; ++k) {
        if (act)
#pragma unroll
            for (int e = 0; e < 7; ++e) pd[size_t(slot) * per + i * 7 + e] = acc[k][e];
        __syncthreads();
        for (int e = t; e < PB * NP1 * 7; e += int(blockDim.x)) {
            const int s2 = e / (NP1 * 7), r = e % (NP1 * 7), n = r / 7, cc = r % 7;
            if (p0 + s2 >= P) continue;
            const double *b = pd + size_t(s2) * per;
            const double *w = swl + n * c.Q;
            double sum = 0.0;
            for (int q = 0; q < c.Q; ++q) sum += w[q] * b[q * 7 + cc];
            pd[size_t(s2) * per + c.Q * 7 + (n * NP1 + k) * 7 + cc] = sum;
        }
        __syncthreads();
    }
    for (int e = t; e < PB * st * st; e += int(blockDim.x)) {
        const int s3 = e / (st * st), r = e % (st * st);
        if (p0 + s3 >= P) continue;
        const int m3 = pairs[2 * s3], mp3 = pairs[2 * s3 + 1];
        const int row = r / st, col = r % st;
        const int n = row / 3, a = row % 3, k = col / 3, b = col % 3;
        const double *o = pd + size_t(s3) * per + c.Q * 7 + (n * NP1 + k) * 7;
        const double v = o[sym_index(a, b)] + (a == b ? o[0] : 0.0);
        // Theta^{n,k}_{m,mp} at (m st + row, mp st + col); its transpose,
        // Theta^{k,n}_{mp,m}, is the mirror entry of the symmetric matrix
        put_sym(W, c.nt, m3 * st + row, mp3 * st + col, v);
    }
}

// Moments for Q > 64: one 64-thread block per ordered pair (m, mp), blocks
// with m >= mp return at once; each thread takes outer points i, i + 64, ...
// and keeps their sums in LDS ([Q][NP1][7], then out[NP1][NP1][7]).
template <int NP1>
__global__ __launch_bounds__(64) void k_theta_wide(const double *__restrict__ X, const double *__restrict__ p,
                                                   Consts c, const double *__restrict__ sq,
                                                   const double *__restrict__ wl, double *__restrict__ W)
{
    const int m = int(blockIdx.x) / c.M, mp = int(blockIdx.x) % c.M;
    const int st = 3 * NP1;
    if (m >= mp) return;
    extern __shared__ double sh[];
    const double xm[3] = {X[3 * m], X[3 * m + 1], X[3 * m + 2]};
    const double pm[3] = {p[3 * m], p[3 * m + 1], p[3 * m + 2]};
    const double xn[3] = {X[3 * mp], X[3 * mp + 1], X[3 * mp + 2]};
    const double pn[3] = {p[3 * mp], p[3 * mp + 1], p[3 * mp + 2]};
    const double h = 0.5 * c.r * c.r;
    double acc[NP1][7];
    double *out = sh + size_t(c.Q) * NP1 * 7;
    for (int i = threadIdx.x; i < c.Q; i += 64) {
        moment_point<NP1>(i, xm, pm, xn, pn, h, c, sq, wl, acc);
#pragma unroll
        for (int k = 0; k < NP1; ++k)
#pragma unroll
            for (int e = 0; e < 7; ++e) sh[(size_t(i) * NP1 + k) * 7 + e] = acc[k][e];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < NP1 * NP1 * 7; e += 64) {
        const int n = e / (NP1 * 7), k = (e / 7) % NP1, cc = e % 7;
        double s = 0.0;
        for (int i = 0; i < c.Q; ++i) s += wl[n * c.Q + i] * sh[(size_t(i) * NP1 + k) * 7 + cc];
        out[e] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < st * st; e += 64) {
        const int row = e / st, col = e % st;
        const int n = row / 3, a = row % 3, k = col / 3, b = col % 3;
        const double *o = out + (n * NP1 + k) * 7;
        const double v = o[sym_index(a, b)] + (a == b ? o[0] : 0.0);
        put_sym(W, c.nt, m * st + row, mp * st + col, v);
    }
}

// Partial products of the packed symmetric matrix.  Workgroup w takes a
// chunk of up to SG consecutive stored tiles of one tile row i, (i, j0) ..
// (i, j0 + ng - 1) (ch[w] = (i, j0, ng, slot)); lane l owns column l of a
// tile, wave v its rows 16 v .. 16 v + 15.  Row sums W_ij x_j build up in
// registers over the chunk and go to part[slot][rows of block i], slot =
// i + (j0 - i)/SG; column sums W_ij^T x_i of each off-diagonal tile go to
// part[i][rows of block j].  For the rows of block b the slots 0 .. b - 1
// hold column sums and b .. b + ceil((nt - b)/SG) - 1 row-sum chunks, each
// written exactly once.  x entries beyond D read as zero.
constexpr int SG = 8;          // tiles per workgroup

__global__ __launch_bounds__(256) void k_symv(const double *__restrict__ W, const double *__restrict__ x,
                                              double *__restrict__ part, const int4 *__restrict__ ch, int D, int nt)
{
    const int4 cw = ch[blockIdx.x];
    const int i = cw.x, j0 = cw.y, ng = cw.z, slot = cw.w;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const size_t ntT = size_t(nt) * TS;
    const double *tile = W + tile_base(i, j0, nt) + size_t(wv * 16) * TS + lane;
    double xr[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int ri = i * TS + wv * 16 + k;
        xr[k] = ri < D ? x[ri] : 0.0;
    }
    __shared__ double cs[SG][4][TS];
    double rp[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) rp[k] = 0.0;
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = tile[k * TS];
    for (int g = 0; g < ng; ++g) {
        const int j = j0 + g;
        const int cj = j * TS + lane;
        const double xc = cj < D ? x[cj] : 0.0;
        double col = 0.0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            col = fma(v[k], xr[k], col);
            rp[k] = fma(v[k], xc, rp[k]);
        }
        cs[g][wv][lane] = col;
        if (g + 1 < ng) {
            tile += TS * TS;
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = tile[k * TS];
        }
    }
    // row sums over the lanes: halve the values held per lane while pairing
    // lanes 32, 16, 8, 4 apart, then add over the last two lane bits; lane l
    // ends with the sum of row 16 v + 8 b5 + 4 b4 + 2 b3 + b2 (b: bits of l)
    const int b5 = (lane >> 5) & 1, b4 = (lane >> 4) & 1, b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double send = b5 ? rp[k] : rp[k + 8], keep = b5 ? rp[k + 8] : rp[k];
        rp[k] = keep + __shfl_xor(send, 32, 64);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double send = b4 ? rp[k] : rp[k + 4], keep = b4 ? rp[k + 4] : rp[k];
        rp[k] = keep + __shfl_xor(send, 16, 64);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const double send = b3 ? rp[k] : rp[k + 2], keep = b3 ? rp[k + 2] : rp[k];
        rp[k] = keep + __shfl_xor(send, 8, 64);
    }
    {
        const double send = b2 ? rp[0] : rp[1], keep = b2 ? rp[1] : rp[0];
        rp[0] = keep + __shfl_xor(send, 4, 64);
    }
    double rs = rp[0] + __shfl_xor(rp[0], 2, 64);
    rs = rs + __shfl_xor(rs, 1, 64);
    if ((lane & 3) == 0) {
        const int r = wv * 16 + 8 * b5 + 4 * b4 + 2 * b3 + b2;
        part[size_t(slot) * ntT + size_t(i) * TS + r] = rs;
    }
    __syncthreads();
    // column sums of the off-diagonal tiles, the four waves' parts in order
    for (int g = wv; g < ng; g += 4) {
        const int j = j0 + g;
        if (j == i) continue;
        part[size_t(i) * ntT + size_t(j) * TS + lane] = (cs[g][0][lane] + cs[g][1][lane]) + (cs[g][2][lane] + cs[g][3][lane]);
    }
}

// y[R] = sum over the partial sums of row R (block b = R / TS): slots
// 0 .. ns - 1, ns = b + ceil((nt - b)/SG).  One workgroup per block of 64
// rows; wave w adds the slots w, w + 4, w + 8, ... (independent loads, four
// accumulators), the four waves' sums are then added in order.
__global__ __launch_bounds__(256) void k_symv_sum(const double *__restrict__ part, double *__restrict__ y, int D,
                                                  int nt)
{
    const int b = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int r = b * TS + lane;
    const int ns = b + (nt - b + SG - 1) / SG;
    const size_t ntT = size_t(nt) * TS;
    const double *pc = part + r;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int t = wv;
    for (; t + 12 < ns; t += 16) {
        a0 += pc[size_t(t) * ntT];
        a1 += pc[size_t(t + 4) * ntT];
        a2 += pc[size_t(t + 8) * ntT];
        a3 += pc[size_t(t + 12) * ntT];
    }
    for (; t < ns; t += 4) a0 += pc[size_t(t) * ntT];
    __shared__ double ws[4][TS];
    ws[wv][lane] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (wv == 0 && r < D) y[r] = (ws[0][lane] + ws[1][lane]) + (ws[2][lane] + ws[3][lane]);
}

// the chunks of k_symv for nt tiles per side: (i, j0, ng, slot) per workgroup
static std::vector<int4> symv_chunks(int nt)
{
    std::vector<int4> out;
    for (int i = 0; i < nt; ++i)
        for (int j0 = i, c = 0; j0 < nt; j0 += SG, ++c) out.push_back(make_int4(i, j0, std::min(SG, nt - j0), i + c));
    return out;
}

static size_t symv_chunk_count(int nt)
{
    size_t n = 0;
    for (int i = 0; i < nt; ++i) n += size_t((nt - i + SG - 1) / SG);
    return n;
}

// per-fiber 3x3 blocks: Lambda = d (I + p p^T) + 2 (I - p p^T), K = I + p p^T
__device__ __forceinline__ void blocks(const double *p, double d, double lam[3][3], double K[3][3], double pp[3][3])
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            const double ab = p[a] * p[b], id = a == b ? 1.0 : 0.0;
            pp[a][b] = ab;
            K[a][b] = id + ab;
            lam[a][b] = d * (id + ab) + 2.0 * (id - ab);
        }
}

// L_n = -2 sum_{i<=n} 1/i: eigenvalue of the finite-part operator on P_n
__device__ __forceinline__ double kbar_eig(int n)
{
    double s = 0.0;
    for (int i = 1; i <= n; ++i) s += 1.0 / double(i);
    return -2.0 * s;
}

// Rows (m, n >= 1) of the system operator from x and z = W x:
//   n >= 2: (Lambda + L_n K) x_n + c_n z_n
//   n  = 1: (I - p p^T) x_1 + p p^T [(Lambda + L_1 K) x_1 + c_1 z_1]
// c_n = (2n + 1)/(2l); rows n = 0 set to zero.  One thread per (m, n).
__global__ __launch_bounds__(256) void k_apply(const double *__restrict__ x, const double *__restrict__ z,
                                               double *__restrict__ y, const double *__restrict__ p, Consts c)
{
    const int t = int(blockIdx.x * blockDim.x + threadIdx.x);
    const int NP1 = c.N + 1;
    if (t >= c.M * NP1) return;
    const int m = t / NP1, n = t % NP1;
    double *yo = y + size_t(3) * t;
    if (n == 0) {
        yo[0] = yo[1] = yo[2] = 0.0;
        return;
    }
    double lam[3][3], K[3][3], pp[3][3];
    blocks(p + 3 * m, c.d, lam, K, pp);
    const double Ln = kbar_eig(n), cn = (2.0 * n + 1.0) / (2.0 * c.l);
    const double *xi = x + size_t(3) * t, *zi = z + size_t(3) * t;
    double v[3];
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int b = 0; b < 3; ++b) s += (lam[a][b] + Ln * K[a][b]) * xi[b];
        v[a] = s + cn * zi[a];
    }
    if (n >= 2) {
        for (int a = 0; a < 3; ++a) yo[a] = v[a];
    } else {
        const double pv = p[3 * m] * v[0] + p[3 * m + 1] * v[1] + p[3 * m + 2] * v[2];
        const double px = p[3 * m] * xi[0] + p[3 * m + 1] * xi[1] + p[3 * m + 2] * xi[2];
        for (int a = 0; a < 3; ++a) yo[a] = (xi[a] - p[3 * m + a] * px) + p[3 * m + a] * pv;
    }
}

// Block-Jacobi preconditioner: out_{m,n} = B_{m,n}^{-1} in_{m,n} with the
// self blocks of the operator, all of the form alpha I + beta p p^T:
//   n >= 2: Lambda + L_n K = (d + 2 + L_n) I + (d - 2 + L_n) p p^T,
//   n  = 1: (I - p p^T) + p p^T (Lambda + L_1 K) = I + (2 d + 2 L_1 - 1) p p^T,
// inverted in closed form, (alpha I + beta p p^T)^-1 =
// (I - beta/(alpha + beta) p p^T)/alpha.  GMRES runs on the right-
// preconditioned operator A B^-1; the self part then is the identity and
// the iteration count reflects the interactions only.
__global__ __launch_bounds__(256) void k_precond(const double *__restrict__ in, double *__restrict__ out,
                                                 const double *__restrict__ p, Consts c)
{
    const int t = int(blockIdx.x * blockDim.x + threadIdx.x);
    const int NP1 = c.N + 1;
    if (t >= c.M * NP1) return;
    const int m = t / NP1, n = t % NP1;
    const double *xi = in + size_t(3) * t;
    double *yo = out + size_t(3) * t;
    if (n == 0) {
        yo[0] = yo[1] = yo[2] = 0.0;
        return;
    }
    const double Ln = kbar_eig(n);
    const double alpha = n == 1 ? 1.0 : c.d + 2.0 + Ln;
    const double beta = n == 1 ? 2.0 * c.d + 2.0 * Ln - 1.0 : c.d - 2.0 + Ln;
    const double *pm = p + 3 * m;
    const double px = pm[0] * xi[0] + pm[1] * xi[1] + pm[2] * xi[2];
    const double f = beta / (alpha + beta);
    for (int a = 0; a < 3; ++a) yo[a] = (xi[a] - f * px * pm[a]) / alpha;
}

// the known part of the force as a vector of the (m, k, b) layout:
// F_m/(2l) in the k = 0 entries, zero elsewhere
__global__ __launch_bounds__(256) void k_known(double *__restrict__ v, const double *__restrict__ F, Consts c)
{
    const int e = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= c.D) return;
    const int b = e % 3, k = (e / 3) % (c.N + 1), m = e / (3 * (c.N + 1));
    v[e] = k == 0 ? F[3 * m + b] / (2.0 * c.l) : 0.0;
}

// right-hand side from z0 = W [F/(2l); 0]:
//   n = 1: 3/(2 l^2) M x p - c_1 p p^T z0_1;  n >= 2: -c_n z0_n;  n = 0: 0
__global__ __launch_bounds__(256) void k_rhs(const double *__restrict__ z0, double *__restrict__ b,
                                             const double *__restrict__ p, const double *__restrict__ Mt, Consts c)
{
    const int t = int(blockIdx.x * blockDim.x + threadIdx.x);
    const int NP1 = c.N + 1;
    if (t >= c.M * NP1) return;
    const int m = t / NP1, n = t % NP1;
    double *bo = b + size_t(3) * t;
    const double *zi = z0 + size_t(3) * t;
    if (n == 0) {
        bo[0] = bo[1] = bo[2] = 0.0;
        return;
    }
    const double cn = (2.0 * n + 1.0) / (2.0 * c.l);
    if (n >= 2) {
        for (int a = 0; a < 3; ++a) bo[a] = -cn * zi[a];
        return;
    }
    const double *pm = p + 3 * m, *mm = Mt + 3 * m;
    const double mxp[3] = {mm[1] * pm[2] - mm[2] * pm[1], mm[2] * pm[0] - mm[0] * pm[2], mm[0] * pm[1] - mm[1] * pm[0]};
    const double pz = pm[0] * zi[0] + pm[1] * zi[1] + pm[2] * zi[2];
    const double tq = 3.0 / (2.0 * c.l * c.l);
    for (int a = 0; a < 3; ++a) bo[a] = tq * mxp[a] - cn * pm[a] * pz;
}

// velocities from z = W [F/(2l); a] (rows n = 0: int U ds, n = 1: int U P_1 ds):
//   dx/dt = (Lambda F + z_0) / (8 pi mu L)
//   dp/dt = 3/(2 pi mu L^3) [d M x p + (I - p p^T) l z_1]
__global__ __launch_bounds__(256) void k_velocity(const double *__restrict__ z, const double *__restrict__ p,
                                                  const double *__restrict__ F, const double *__restrict__ Mt,
                                                  double *__restrict__ V, double *__restrict__ Pd, Consts c)
{
    const int m = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (m >= c.M) return;
    const int NP1 = c.N + 1;
    double lam[3][3], K[3][3], pp[3][3];
    blocks(p + 3 * m, c.d, lam, K, pp);
    const double *z0 = z + size_t(3) * (m * NP1), *z1 = z0 + 3;
    const double *pm = p + 3 * m, *mm = Mt + 3 * m, *f = F + 3 * m;
    const double kv = 1.0 / (8.0 * M_PI * c.mu * c.L);
    const double kw = 3.0 / (2.0 * M_PI * c.mu * c.L * c.L * c.L);
    const double mxp[3] = {mm[1] * pm[2] - mm[2] * pm[1], mm[2] * pm[0] - mm[0] * pm[2], mm[0] * pm[1] - mm[1] * pm[0]};
    const double pz = pm[0] * z1[0] + pm[1] * z1[1] + pm[2] * z1[2];
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int b = 0; b < 3; ++b) s += lam[a][b] * f[b];
        V[3 * m + a] = kv * (s + z0[a]);
        Pd[3 * m + a] = kw * (c.d * mxp[a] + c.l * (z1[a] - pm[a] * pz));
    }
}

// ------------------------------------------------------------------ GMRES pieces
// h[j] = <V_j, w> for j < nj in two passes with a fixed summation order:
// workgroup (j, p) sums chunk p of DP chunks of the vectors into
// part[j DP + p]; k_dots_sum adds the DP partial sums of each j in order.
constexpr int DP = 16;

__global__ __launch_bounds__(256) void k_dots(const double *__restrict__ Vb, const double *__restrict__ w,
                                              double *__restrict__ part, int D)
{
    const int j = blockIdx.y, pc = blockIdx.x;
    const int chunk = (D + DP - 1) / DP, e0 = pc * chunk, e1 = min(D, e0 + chunk);
    const double *v = Vb + size_t(j) * D;
    double s = 0.0;
    for (int e = e0 + int(threadIdx.x); e < e1; e += 256) s += v[e] * w[e];
    __shared__ double red[4];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[j * DP + pc] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(64) void k_dots_sum(const double *__restrict__ part, double *__restrict__ h, int nj)
{
    const int j = int(threadIdx.x);
    if (j >= nj) return;
    double s = 0.0;
    for (int p = 0; p < DP; ++p) s += part[j * DP + p];
    h[j] = s;
}

// w -= sum_{j < nj} h[j] V_j; acc[j] += h[j] (the column of H)
__global__ __launch_bounds__(256) void k_orth(const double *__restrict__ Vb, double *__restrict__ w,
                                              const double *__restrict__ h, int nj, int D)
{
    const int e = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= D) return;
    double s = w[e];
    for (int j = 0; j < nj; ++j) s -= h[j] * Vb[size_t(j) * D + e];
    w[e] = s;
}

// single thread: H column i += correction; norm of w -> H[i+1][i]; Givens
// rotations on the column; residual |g[i+1]| into res[0]
__global__ void k_hcol(double *__restrict__ H, const double *__restrict__ h1, const double *__restrict__ h2,
                       const double *__restrict__ nrm, double *__restrict__ cs, double *__restrict__ sn,
                       double *__restrict__ g, double *__restrict__ res, int i)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double col[MAXR + 1];
    for (int j = 0; j <= i; ++j) col[j] = h1[j] + h2[j];
    col[i + 1] = sqrt(nrm[0]);
    for (int j = 0; j < i; ++j) {
        const double a = cs[j] * col[j] + sn[j] * col[j + 1];
        const double b = -sn[j] * col[j] + cs[j] * col[j + 1];
        col[j] = a;
        col[j + 1] = b;
    }
    const double a = col[i], b = col[i + 1];
    const double rr = sqrt(a * a + b * b);
    const double c = rr > 0.0 ? a / rr : 1.0, s = rr > 0.0 ? b / rr : 0.0;
    cs[i] = c;
    sn[i] = s;
    col[i] = rr;
    col[i + 1] = 0.0;
    g[i + 1] = -s * g[i];
    g[i] = c * g[i];
    for (int j = 0; j <= i; ++j) H[j * MAXR + i] = col[j];
    res[0] = fabs(g[i + 1]);
}

// V_{i+1} = w / sqrt(nrm) (zero when the Krylov space is exhausted)
__global__ __launch_bounds__(256) void k_normalize(const double *__restrict__ w, double *__restrict__ v,
                                                   const double *__restrict__ nrm, int D)
{
    const int e = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= D) return;
    const double n = sqrt(nrm[0]);
    v[e] = n > 0.0 ? w[e] / n : 0.0;
}

// r = b - y; nrm = <r, r> computed separately; g = (|r|, 0, ...)
__global__ __launch_bounds__(256) void k_residual(const double *__restrict__ b, const double *__restrict__ y,
                                                  double *__restrict__ r, int D)
{
    const int e = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (e < D) r[e] = b[e] - y[e];
}

__global__ void k_gstart(double *__restrict__ g, const double *__restrict__ nrm, double *__restrict__ res)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        g[0] = sqrt(nrm[0]);
        res[0] = g[0];
    }
}

// back substitution H y = g over k columns
__global__ void k_backsolve(const double *__restrict__ H, const double *__restrict__ g, double *__restrict__ y,
                            int k)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int i = k - 1; i >= 0; --i) {
        double s = g[i];
        for (int j = i + 1; j < k; ++j) s -= H[i * MAXR + j] * y[j];
        const double d = H[i * MAXR + i];
        y[i] = d != 0.0 ? s / d : 0.0;
    }
}

// out = sum_{j < k} y_j V_j
__global__ __launch_bounds__(256) void k_lincomb(double *__restrict__ out, const double *__restrict__ Vb,
                                                 const double *__restrict__ y, int k, int D)
{
    const int e = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= D) return;
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += y[j] * Vb[size_t(j) * D + e];
    out[e] = s;
}

// out = a + b
__global__ __launch_bounds__(256) void k_add(const double *a, const double *b, double *out, int D)
{
    const int e = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (e < D) out[e] = a[e] + b[e];
}

// GMRES start of a time step: the linear extrapolation 2 a_n - a_{n-1} of
// the last two solutions (x holds a_n, xh a_{n-1}); xh takes a_n
__global__ __launch_bounds__(256) void k_extrap(double *__restrict__ x, double *__restrict__ xh, int D)
{
    const int e = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (e >= D) return;
    const double a = x[e];
    x[e] = 2.0 * a - xh[e];
    xh[e] = a;
}

// Adams-Bashforth 2 (Euler when first), p renormalised
__global__ __launch_bounds__(256) void k_advance(double *__restrict__ X, double *__restrict__ p,
                                                 const double *__restrict__ V, const double *__restrict__ Pd,
                                                 double *__restrict__ Vp, double *__restrict__ Pp, int M, double dt,
                                                 int first)
{
    const int m = int(blockIdx.x * blockDim.x + threadIdx.x);
    if (m >= M) return;
    double q[3];
    for (int a = 0; a < 3; ++a) {
        const double v = V[3 * m + a], w = Pd[3 * m + a];
        const double dv = first ? v : 1.5 * v - 0.5 * Vp[3 * m + a];
        const double dw = first ? w : 1.5 * w - 0.5 * Pp[3 * m + a];
        X[3 * m + a] += dt * dv;
        q[a] = p[3 * m + a] + dt * dw;
        Vp[3 * m + a] = v;
        Pp[3 * m + a] = w;
    }
    const double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    for (int a = 0; a < 3; ++a) p[3 * m + a] = q[a] / n;
}

}  // namespace sbfk

using namespace sbfk;

struct sbf_ctx {
    sbf_params p{};
    std::string err;
    hipStream_t st = nullptr;
    bool own_stream = false;
    Consts c{};
    int M = 0, Dmax = 0;
    // device
    double *X = nullptr, *pd = nullptr, *F = nullptr, *Mt = nullptr;
    double *sq = nullptr, *wl = nullptr;   // quadrature nodes; weights times P_k at the nodes
    double *W = nullptr;                   // packed upper triangle of the moment matrix
    double *part = nullptr;                // [nt][nt TS] partial sums of a product with W
    int4 *chunks = nullptr;                // work list of the product kernel
    double *dpart = nullptr;               // [MAXR][DP] partial dot products
    unsigned nchunks = 0;
    double *x = nullptr, *b = nullptr, *r = nullptr, *w = nullptr, *y = nullptr, *kn = nullptr, *z = nullptr;
    double *t = nullptr, *u = nullptr;     // preconditioned vectors
    double *xh = nullptr;                   // the solution of the previous time step
    int nsol = 0;                           // solutions of time steps since the fibers were set
    double *Vb = nullptr;                   // [restart + 1][D]
    double *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *h1 = nullptr, *h2 = nullptr, *ys = nullptr;
    double *nrm = nullptr, *res = nullptr;  // scalars
    double *resh = nullptr;                 // pinned host copies of the residual, one per iteration
    hipEvent_t rev[MAXR] = {};              // recorded after each copy
    double *V = nullptr, *Pd = nullptr, *Vp = nullptr, *Pp = nullptr;
    bool first = true, solved = false;
    // event timing: pairs recorded around the moment kernel and each GEMV
    bool timing = false;
    std::vector<hipEvent_t> ev;
    size_t ev_used = 0;
    std::vector<int> ev_kind;    // 0 moments, 1 GEMV
    double t_theta = 0.0, t_gemv = 0.0;
    int64_t n_theta = 0, n_gemv = 0;
    int iters = 0;
    double relres = 0.0;
    int64_t steps = 0;
};

static lbm_status sfail(sbf_ctx *c, lbm_status s, const std::string &m)
{
    if (c) c->err = m;
    return s;
}

#define SCHK(c, call)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return sfail((c), e_ == hipErrorOutOfMemory ? LBM_E_NOMEM : LBM_E_HIP,                     \
                         std::string(#call) + ": " + hipGetErrorString(e_));                           \
    } while (0)

static inline unsigned nblk(size_t n) { return unsigned((n + 255) / 256); }

// launch of the moment kernel for the compile-time number of modes
template <int NP1>
static hipError_t theta_t(sbf_ctx *c)
{
    const int Q = c->c.Q;
    if (c->M < 2) return hipSuccess;
    if (Q > 64) {
        const size_t lds = (size_t(Q) * NP1 * 7 + size_t(NP1) * NP1 * 7) * sizeof(double);
        hipLaunchKernelGGL((k_theta_wide<NP1>), dim3(unsigned(c->M) * unsigned(c->M)), dim3(64), lds, c->st, c->X,
                           c->pd, c->c, c->sq, c->wl, c->W);
        return hipGetLastError();
    }
    // pairs per workgroup: the most lanes busy (PB Q over whole waves), then
    // the most pairs, within 64 KiB of LDS
    const size_t per_pair = (size_t(Q) * 7 + size_t(NP1) * NP1 * 7) * sizeof(double);
    const size_t fixed = size_t(NP1) * Q * sizeof(double);   // the weights; (m, m') pairs below
    int pb = 1;
    double best = 0.0;
    for (int k = 1; k * Q <= 256 && fixed + size_t((k + 1) / 2 * 2) * 8 + size_t(k) * per_pair <= 65536; ++k) {
        const double use = double(k * Q) / double(((k * Q + 63) / 64) * 64);
        if (use >= best) {
            best = use;
            pb = k;
        }
    }
    const unsigned threads = unsigned(((pb * Q + 63) / 64) * 64);
    const long long P = (long long)c->M * (c->M - 1) / 2;
    const size_t lds = fixed + size_t((pb + 1) / 2 * 2) * sizeof(double) + size_t(pb) * per_pair;
    hipLaunchKernelGGL((k_theta<NP1>), dim3(unsigned((P + pb - 1) / pb)), dim3(threads), lds, c->st, c->X, c->pd,
                       c->c, c->sq, c->wl, c->W, pb, P);
    return hipGetLastError();
}

static hipError_t launch_theta(sbf_ctx *c)
{
    switch (c->c.N + 1) {
    case 2: return theta_t<2>(c);
    case 3: return theta_t<3>(c);
    case 4: return theta_t<4>(c);
    case 5: return theta_t<5>(c);
    case 6: return theta_t<6>(c);
    case 7: return theta_t<7>(c);
    case 8: return theta_t<8>(c);
    default: return theta_t<9>(c);
    }
}

// an event pair around the next launch when timing (kind 0: moments, 1: GEMV)
static hipError_t mark(sbf_ctx *c, int kind, bool begin)
{
    if (!c->timing) return hipSuccess;
    if (begin) {
        while (c->ev.size() < c->ev_used + 2) {
            hipEvent_t e;
            hipError_t r = hipEventCreate(&e);
            if (r != hipSuccess) return r;
            c->ev.push_back(e);
        }
        c->ev_kind.resize(c->ev.size() / 2 + 1);
        c->ev_kind[c->ev_used / 2] = kind;
    }
    return hipEventRecord(c->ev[c->ev_used++], c->st);
}

// after a synchronisation: add the recorded pairs to the totals
static hipError_t collect(sbf_ctx *c)
{
    for (size_t i = 0; i + 1 < c->ev_used; i += 2) {
        float ms = 0.0f;
        hipError_t r = hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]);
        if (r != hipSuccess) return r;
        if (c->ev_kind[i / 2] == 0) {
            c->t_theta += ms;
            c->n_theta += 1;
        } else {
            c->t_gemv += ms;
            c->n_gemv += 1;
        }
    }
    c->ev_used = 0;
    return hipSuccess;
}

static hipError_t gemv(sbf_ctx *c, const double *xin, double *yout)
{
    hipError_t e = mark(c, 1, true);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_symv, dim3(c->nchunks), dim3(256), 0, c->st, c->W, xin, c->part, c->chunks, c->c.D,
                       c->c.nt);
    hipLaunchKernelGGL(k_symv_sum, dim3(unsigned(c->c.nt)), dim3(256), 0, c->st, c->part, yout, c->c.D, c->c.nt);
    e = hipGetLastError();
    return e != hipSuccess ? e : mark(c, 1, false);
}

// y = A x (system operator)
static hipError_t apply(sbf_ctx *c, const double *xin, double *yout)
{
    hipError_t e = gemv(c, xin, c->z);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_apply, dim3(nblk(size_t(c->M) * (c->c.N + 1))), dim3(256), 0, c->st, xin, c->z, yout,
                       c->pd, c->c);
    return hipGetLastError();
}

// out = B^-1 in (block-Jacobi)
static hipError_t precond(sbf_ctx *c, const double *in, double *out)
{
    hipLaunchKernelGGL(k_precond, dim3(nblk(size_t(c->M) * (c->c.N + 1))), dim3(256), 0, c->st, in, out, c->pd,
                       c->c);
    return hipGetLastError();
}

// nrm = <v, v>
// h[0 .. nj) = <V_j, w> for the nj vectors starting at Vb
static hipError_t dots(sbf_ctx *c, const double *Vb, const double *w, double *h, int nj)
{
    hipLaunchKernelGGL(k_dots, dim3(DP, unsigned(nj)), dim3(256), 0, c->st, Vb, w, c->dpart, c->c.D);
    hipLaunchKernelGGL(k_dots_sum, dim3(1), dim3(64), 0, c->st, c->dpart, h, nj);
    return hipGetLastError();
}

static hipError_t dot_self(sbf_ctx *c, const double *v) { return dots(c, v, v, c->nrm, 1); }

static lbm_status read_scalar(sbf_ctx *c, const double *dptr, double *out)
{
    SCHK(c, hipMemcpyAsync(out, dptr, sizeof(double), hipMemcpyDeviceToHost, c->st));
    SCHK(c, hipStreamSynchronize(c->st));
    SCHK(c, collect(c));
    return LBM_OK;
}

// moments, right-hand side, GMRES (right block-Jacobi preconditioning, from
// the previous solution), velocities
static lbm_status do_solve(sbf_ctx *c)
{
    const int D = c->c.D;
    const unsigned gd = nblk(size_t(D));
    SCHK(c, mark(c, 0, true));
    SCHK(c, launch_theta(c));
    SCHK(c, mark(c, 0, false));
    hipLaunchKernelGGL(k_known, dim3(gd), dim3(256), 0, c->st, c->kn, c->F, c->c);
    SCHK(c, hipGetLastError());
    SCHK(c, gemv(c, c->kn, c->z));
    hipLaunchKernelGGL(k_rhs, dim3(nblk(size_t(c->M) * (c->c.N + 1))), dim3(256), 0, c->st, c->z, c->b, c->pd,
                       c->Mt, c->c);
    SCHK(c, hipGetLastError());
    SCHK(c, dot_self(c, c->b));
    double bn2 = 0.0;
    lbm_status s = read_scalar(c, c->nrm, &bn2);
    if (s != LBM_OK) return s;
    const double bnorm = std::sqrt(bn2);
    const int R = c->p.gmres_restart;
    int it = 0;
    double rel = 0.0;
    bool conv = false;
    if (bnorm == 0.0) {
        SCHK(c, hipMemsetAsync(c->x, 0, size_t(D) * sizeof(double), c->st));
        conv = true;
    }
    while (!conv && it < c->p.gmres_maxit) {
        // r = b - A x, V_0 = r/|r|, g = (|r|, 0, ...)
        SCHK(c, apply(c, c->x, c->y));
        hipLaunchKernelGGL(k_residual, dim3(gd), dim3(256), 0, c->st, c->b, c->y, c->r, D);
        SCHK(c, hipGetLastError());
        SCHK(c, dot_self(c, c->r));
        hipLaunchKernelGGL(k_gstart, dim3(1), dim3(64), 0, c->st, c->g, c->nrm, c->res);
        hipLaunchKernelGGL(k_normalize, dim3(gd), dim3(256), 0, c->st, c->r, c->Vb, c->nrm, D);
        SCHK(c, hipGetLastError());
        double r0 = 0.0;
        if ((s = read_scalar(c, c->res, &r0)) != LBM_OK) return s;
        rel = r0 / bnorm;
        if (rel <= c->p.gmres_tol) {
            conv = true;
            break;
        }
        int k = 0;
        for (int i = 0; i < R && it < c->p.gmres_maxit; ++i) {
            double *vi = c->Vb + size_t(i) * D, *vn = c->Vb + size_t(i + 1) * D;
            SCHK(c, precond(c, vi, c->t));
            SCHK(c, apply(c, c->t, c->w));
            // classical Gram-Schmidt, twice
            SCHK(c, dots(c, c->Vb, c->w, c->h1, i + 1));
            hipLaunchKernelGGL(k_orth, dim3(gd), dim3(256), 0, c->st, c->Vb, c->w, c->h1, i + 1, D);
            SCHK(c, dots(c, c->Vb, c->w, c->h2, i + 1));
            hipLaunchKernelGGL(k_orth, dim3(gd), dim3(256), 0, c->st, c->Vb, c->w, c->h2, i + 1, D);
            SCHK(c, hipGetLastError());
            SCHK(c, dot_self(c, c->w));
            hipLaunchKernelGGL(k_hcol, dim3(1), dim3(64), 0, c->st, c->H, c->h1, c->h2, c->nrm, c->cs, c->sn, c->g,
                               c->res, i);
            hipLaunchKernelGGL(k_normalize, dim3(gd), dim3(256), 0, c->st, c->w, vn, c->nrm, D);
            SCHK(c, hipGetLastError());
            // the residual of this iteration to pinned host memory; the host
            // tests the previous iteration's while this one runs, so the
            // stream never drains for the test (at most one iteration more
            // than needed, which only lowers the residual)
            SCHK(c, hipMemcpyAsync(c->resh + i, c->res, sizeof(double), hipMemcpyDeviceToHost, c->st));
            SCHK(c, hipEventRecord(c->rev[i], c->st));
            ++it;
            k = i + 1;
            if (i >= 1) {
                SCHK(c, hipEventSynchronize(c->rev[i - 1]));
                rel = c->resh[i - 1] / bnorm;
                if (rel <= c->p.gmres_tol) {
                    conv = true;
                    break;
                }
            }
        }
        if (!conv && k > 0) {
            SCHK(c, hipEventSynchronize(c->rev[k - 1]));
            rel = c->resh[k - 1] / bnorm;
            conv = rel <= c->p.gmres_tol;
        }
        // x += B^-1 sum_j y_j V_j
        hipLaunchKernelGGL(k_backsolve, dim3(1), dim3(64), 0, c->st, c->H, c->g, c->ys, k);
        hipLaunchKernelGGL(k_lincomb, dim3(gd), dim3(256), 0, c->st, c->t, c->Vb, c->ys, k, D);
        SCHK(c, hipGetLastError());
        SCHK(c, precond(c, c->t, c->u));
        hipLaunchKernelGGL(k_add, dim3(gd), dim3(256), 0, c->st, c->x, c->u, c->x, D);
        SCHK(c, hipGetLastError());
    }
    // velocities from W [F/(2l); a]: x (zero k = 0 entries) plus the known part
    hipLaunchKernelGGL(k_known, dim3(gd), dim3(256), 0, c->st, c->kn, c->F, c->c);
    hipLaunchKernelGGL(k_add, dim3(gd), dim3(256), 0, c->st, c->x, c->kn, c->y, D);
    SCHK(c, hipGetLastError());
    SCHK(c, gemv(c, c->y, c->z));
    hipLaunchKernelGGL(k_velocity, dim3(nblk(size_t(c->M))), dim3(256), 0, c->st, c->z, c->pd, c->F, c->Mt, c->V,
                       c->Pd, c->c);
    SCHK(c, hipGetLastError());
    c->iters = it;
    c->relres = rel;
    c->solved = true;
    return conv ? LBM_OK : sfail(c, LBM_E_UNSTABLE, "GMRES did not reach the tolerance");
}

// ====================================================================== ABI
template <typename T>
static hipError_t salloc(T **ptr, size_t n)
{
    *ptr = nullptr;
    return hipMalloc((void **)ptr, std::max<size_t>(n, 1) * sizeof(T));
}

static void release(sbf_ctx *c)
{
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    c->ev.clear();
    double **bufs[] = {&c->X, &c->pd, &c->F, &c->Mt, &c->sq, &c->wl, &c->W, &c->part, &c->dpart, &c->x, &c->xh, &c->b, &c->r,
                       &c->w, &c->y, &c->kn, &c->z, &c->t, &c->u, &c->Vb, &c->H, &c->cs, &c->sn, &c->g, &c->h1, &c->h2,
                       &c->ys, &c->nrm, &c->res, &c->V, &c->Pd, &c->Vp, &c->Pp};
    for (double **b : bufs)
        if (*b) {
            (void)hipFree(*b);
            *b = nullptr;
        }
    if (c->chunks) {
        (void)hipFree(c->chunks);
        c->chunks = nullptr;
    }
    if (c->resh) {
        (void)hipHostFree(c->resh);
        c->resh = nullptr;
    }
    for (hipEvent_t &e : c->rev)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
}

extern "C" {

lbm_status sbf_params_default(sbf_params *p)
{
    if (!p) return LBM_E_ARG;
    std::memset(p, 0, sizeof *p);
    p->max_fibers = 64;
    p->nmodes = 5;
    p->nq = 16;
    p->gmres_restart = 30;
    p->gmres_maxit = 200;
    p->length = 1.0;
    p->eps = 0.1;
    p->mu = 1.0;
    p->gmres_tol = 1e-12;
    return LBM_OK;
}

lbm_status sbf_create(const sbf_params *p, sbf_ctx **out)
{
    if (!p || !out) return LBM_E_ARG;
    *out = nullptr;
    if (p->max_fibers < 1 || p->nmodes < 1 || p->nmodes > MAXN || p->nq < 1 || p->nq > 64 ||
        p->gmres_restart < 1 || p->gmres_restart > MAXR - 1 || p->gmres_maxit < 1)
        return LBM_E_ARG;
    if (!(p->length > 0.0) || !(p->eps > 0.0 && p->eps < 0.5) || !(p->mu > 0.0) || !(p->gmres_tol > 0.0))
        return LBM_E_ARG;
    const size_t lds = size_t(p->nmodes + 1) * 7 * (3 * size_t(p->nq) + size_t(p->nmodes + 1)) * sizeof(double);
    if (lds > 65536) return LBM_E_ARG;
    const double dmax = 3.0 * p->max_fibers * (p->nmodes + 1);
    if (dmax * dmax > 6.0e10) return LBM_E_ARG;   // the packed moment matrix would exceed 240 GB
    sbf_ctx *c = new (std::nothrow) sbf_ctx;
    if (!c) return LBM_E_NOMEM;
    c->p = *p;
    c->st = (hipStream_t)p->stream;
    if (!c->st) {
        if (hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return LBM_E_HIP;
        }
        c->own_stream = true;
    }
    const int N = p->nmodes, Q = 3 * p->nq, Mx = p->max_fibers, R = p->gmres_restart;
    c->Dmax = 3 * Mx * (N + 1);
    const size_t Dm = size_t(c->Dmax);
    const int ntm = (c->Dmax + TS - 1) / TS;
    c->c.N = N;
    c->c.Q = Q;
    c->c.L = p->length;
    c->c.l = 0.5 * p->length;
    c->c.r = p->eps * p->length;
    c->c.d = -std::log(p->eps * p->eps * std::exp(1.0));
    c->c.mu = p->mu;
    hipError_t e = hipSuccess;
    auto A = [&](double **ptr, size_t n) {
        if (e == hipSuccess) e = salloc(ptr, n);
    };
    A(&c->X, 3 * size_t(Mx));
    A(&c->pd, 3 * size_t(Mx));
    A(&c->F, 3 * size_t(Mx));
    A(&c->Mt, 3 * size_t(Mx));
    A(&c->V, 3 * size_t(Mx));
    A(&c->Pd, 3 * size_t(Mx));
    A(&c->Vp, 3 * size_t(Mx));
    A(&c->Pp, 3 * size_t(Mx));
    A(&c->sq, size_t(Q));
    A(&c->wl, size_t(Q) * (N + 1));
    A(&c->W, packed_tiles(ntm) * TS * TS);
    A(&c->part, size_t(ntm) * size_t(ntm) * TS);
    A(&c->dpart, size_t(MAXR) * DP);
    if (e == hipSuccess) e = hipMalloc((void **)&c->chunks, std::max<size_t>(symv_chunk_count(ntm), 1) * sizeof(int4));
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->resh, MAXR * sizeof(double), hipHostMallocDefault);
    for (int i = 0; i < MAXR && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&c->rev[i], hipEventDisableTiming);
    for (double **v : {&c->x, &c->xh, &c->b, &c->r, &c->w, &c->y, &c->kn, &c->z, &c->t, &c->u}) A(v, Dm);
    A(&c->Vb, Dm * size_t(R + 1));
    A(&c->H, size_t(MAXR) * MAXR);
    for (double **v : {&c->cs, &c->sn, &c->g, &c->h1, &c->h2, &c->ys}) A(v, size_t(MAXR + 1));
    A(&c->nrm, 1);
    A(&c->res, 1);
    if (e != hipSuccess) {
        release(c);
        if (c->own_stream) (void)hipStreamDestroy(c->st);
        delete c;
        return e == hipErrorOutOfMemory ? LBM_E_NOMEM : LBM_E_HIP;
    }
    // composite three-point Gauss rule on [-l, l] (nodes +-sqrt(3/5), 0;
    // weights 5/9, 8/9, 5/9 on each sub-interval) and P_0..P_N at its nodes
    std::vector<double> sq(Q), wq(Q), leg(size_t(Q) * (N + 1));
    const double gn[3] = {-std::sqrt(0.6), 0.0, std::sqrt(0.6)}, gw[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
    const double hstep = 2.0 / p->nq;
    for (int i = 0; i < p->nq; ++i)
        for (int k = 0; k < 3; ++k) {
            const double t = -1.0 + hstep * (i + 0.5) + 0.5 * hstep * gn[k];
            const int j = 3 * i + k;
            sq[j] = c->c.l * t;
            wq[j] = c->c.l * 0.5 * hstep * gw[k];
            double p0 = 1.0, p1 = t;
            leg[j] = 1.0;
            if (N >= 1) leg[size_t(Q) + j] = t;
            for (int n = 1; n < N; ++n) {
                const double p2 = ((2 * n + 1) * t * p1 - n * p0) / (n + 1);
                leg[size_t(n + 1) * Q + j] = p2;
                p0 = p1;
                p1 = p2;
            }
        }
    std::vector<double> wl(leg.size());
    for (int k = 0; k <= N; ++k)
        for (int j = 0; j < Q; ++j) wl[size_t(k) * Q + j] = wq[j] * leg[size_t(k) * Q + j];
    if (hipMemcpyAsync(c->sq, sq.data(), Q * sizeof(double), hipMemcpyHostToDevice, c->st) != hipSuccess ||
        hipMemcpyAsync(c->wl, wl.data(), wl.size() * sizeof(double), hipMemcpyHostToDevice, c->st) != hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess) {
        release(c);
        if (c->own_stream) (void)hipStreamDestroy(c->st);
        delete c;
        return LBM_E_HIP;
    }
    *out = c;
    return LBM_OK;
}

lbm_status sbf_destroy(sbf_ctx *c)
{
    if (!c) return LBM_E_ARG;
    (void)hipStreamSynchronize(c->st);
    release(c);
    if (c->own_stream) (void)hipStreamDestroy(c->st);
    delete c;
    return LBM_OK;
}

const char *sbf_last_error(const sbf_ctx *c) { return c ? c->err.c_str() : ""; }

lbm_status sbf_set_fibers(sbf_ctx *c, int32_t m, const double *X, const double *p, const double *F,
                          const double *M)
{
    if (!c) return LBM_E_ARG;
    if (m < 1 || m > c->p.max_fibers || !X || !p) return sfail(c, LBM_E_ARG, "sbf_set_fibers: bad arguments");
    std::vector<double> pn(3 * size_t(m)), zero(3 * size_t(m), 0.0);
    for (int i = 0; i < m; ++i) {
        const double n = std::sqrt(p[3 * i] * p[3 * i] + p[3 * i + 1] * p[3 * i + 1] + p[3 * i + 2] * p[3 * i + 2]);
        if (!(n > 0.0) || !std::isfinite(n)) return sfail(c, LBM_E_ARG, "sbf_set_fibers: zero direction");
        for (int k = 0; k < 3; ++k) pn[3 * i + k] = p[3 * i + k] / n;
    }
    c->M = m;
    c->c.M = m;
    c->c.D = 3 * m * (c->c.N + 1);
    c->c.nt = (c->c.D + TS - 1) / TS;
    const size_t b3 = 3 * size_t(m) * sizeof(double);
    SCHK(c, hipMemcpyAsync(c->X, X, b3, hipMemcpyHostToDevice, c->st));
    SCHK(c, hipMemcpyAsync(c->pd, pn.data(), b3, hipMemcpyHostToDevice, c->st));
    SCHK(c, hipMemcpyAsync(c->F, F ? F : zero.data(), b3, hipMemcpyHostToDevice, c->st));
    SCHK(c, hipMemcpyAsync(c->Mt, M ? M : zero.data(), b3, hipMemcpyHostToDevice, c->st));
    SCHK(c, hipMemsetAsync(c->x, 0, size_t(c->c.D) * sizeof(double), c->st));
    // the diagonal blocks and the padding of the packed matrix stay zero
    SCHK(c, hipMemsetAsync(c->W, 0, packed_tiles(c->c.nt) * TS * TS * sizeof(double), c->st));
    const std::vector<int4> chunks = symv_chunks(c->c.nt);
    c->nchunks = unsigned(chunks.size());
    SCHK(c, hipMemcpyAsync(c->chunks, chunks.data(), chunks.size() * sizeof(int4), hipMemcpyHostToDevice, c->st));
    SCHK(c, hipStreamSynchronize(c->st));
    c->first = true;
    c->solved = false;
    c->steps = 0;
    c->nsol = 0;
    return LBM_OK;
}

lbm_status sbf_solve(sbf_ctx *c)
{
    if (!c) return LBM_E_ARG;
    if (c->M < 1) return sfail(c, LBM_E_STATE, "sbf_solve: no fibers set");
    return do_solve(c);
}

lbm_status sbf_get_velocities(sbf_ctx *c, double *V, double *pdot)
{
    if (!c) return LBM_E_ARG;
    if (!c->solved) return sfail(c, LBM_E_STATE, "no solve since the fibers were set");
    const size_t b3 = 3 * size_t(c->M) * sizeof(double);
    if (V) SCHK(c, hipMemcpyAsync(V, c->V, b3, hipMemcpyDeviceToHost, c->st));
    if (pdot) SCHK(c, hipMemcpyAsync(pdot, c->Pd, b3, hipMemcpyDeviceToHost, c->st));
    SCHK(c, hipStreamSynchronize(c->st));
    return LBM_OK;
}

lbm_status sbf_get_coefficients(sbf_ctx *c, double *a)
{
    if (!c || !a) return LBM_E_ARG;
    if (!c->solved) return sfail(c, LBM_E_STATE, "no solve since the fibers were set");
    std::vector<double> h(size_t(c->c.D));
    SCHK(c, hipMemcpyAsync(h.data(), c->x, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->st));
    SCHK(c, hipStreamSynchronize(c->st));
    const int N = c->c.N;
    for (int m = 0; m < c->M; ++m)
        for (int n = 1; n <= N; ++n)
            for (int b = 0; b < 3; ++b) a[(size_t(m) * N + (n - 1)) * 3 + b] = h[(size_t(m) * (N + 1) + n) * 3 + b];
    return LBM_OK;
}

lbm_status sbf_step(sbf_ctx *c, int64_t n, double dt)
{
    if (!c) return LBM_E_ARG;
    if (n < 0 || !(dt > 0.0)) return sfail(c, LBM_E_ARG, "sbf_step: n >= 0 and dt > 0 required");
    if (c->M < 1) return sfail(c, LBM_E_STATE, "sbf_step: no fibers set");
    for (int64_t s = 0; s < n; ++s) {
        // GMRES starts from the extrapolation of the last two solutions
        // (from the last one after the first step)
        const unsigned gd = nblk(size_t(c->c.D));
        if (c->nsol >= 2) {
            hipLaunchKernelGGL(k_extrap, dim3(gd), dim3(256), 0, c->st, c->x, c->xh, c->c.D);
            SCHK(c, hipGetLastError());
        } else if (c->nsol == 1) {
            SCHK(c, hipMemcpyAsync(c->xh, c->x, size_t(c->c.D) * sizeof(double), hipMemcpyDeviceToDevice, c->st));
        }
        lbm_status st = do_solve(c);
        if (st != LBM_OK) return st;
        c->nsol += 1;
        hipLaunchKernelGGL(k_advance, dim3(nblk(size_t(c->M))), dim3(256), 0, c->st, c->X, c->pd, c->V, c->Pd,
                           c->Vp, c->Pp, c->M, dt, c->first ? 1 : 0);
        SCHK(c, hipGetLastError());
        c->first = false;
        c->steps += 1;
    }
    SCHK(c, hipStreamSynchronize(c->st));
    return LBM_OK;
}

lbm_status sbf_get_state(sbf_ctx *c, double *X, double *p)
{
    if (!c) return LBM_E_ARG;
    const size_t b3 = 3 * size_t(c->M) * sizeof(double);
    if (X) SCHK(c, hipMemcpyAsync(X, c->X, b3, hipMemcpyDeviceToHost, c->st));
    if (p) SCHK(c, hipMemcpyAsync(p, c->pd, b3, hipMemcpyDeviceToHost, c->st));
    SCHK(c, hipStreamSynchronize(c->st));
    return LBM_OK;
}

lbm_status sbf_get_stats(sbf_ctx *c, int32_t *iterations, double *residual, int64_t *steps)
{
    if (!c) return LBM_E_ARG;
    if (iterations) *iterations = c->iters;
    if (residual) *residual = c->relres;
    if (steps) *steps = c->steps;
    return LBM_OK;
}

lbm_status sbf_enable_timing(sbf_ctx *c, int32_t on)
{
    if (!c) return LBM_E_ARG;
    SCHK(c, hipStreamSynchronize(c->st));
    SCHK(c, collect(c));
    c->timing = on != 0;
    if (c->timing) {
        c->t_theta = c->t_gemv = 0.0;
        c->n_theta = c->n_gemv = 0;
    }
    return LBM_OK;
}

lbm_status sbf_get_timing(sbf_ctx *c, double *moments_ms, int64_t *moments_launches, double *gemv_ms,
                          int64_t *gemv_launches)
{
    if (!c) return LBM_E_ARG;
    SCHK(c, hipStreamSynchronize(c->st));
    SCHK(c, collect(c));
    if (moments_ms) *moments_ms = c->t_theta;
    if (moments_launches) *moments_launches = c->n_theta;
    if (gemv_ms) *gemv_ms = c->t_gemv;
    if (gemv_launches) *gemv_launches = c->n_gemv;
    return LBM_OK;
}

}  // extern "C"
