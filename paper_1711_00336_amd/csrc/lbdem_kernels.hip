// HIP kernels (gfx950) of one coupled LBM-DEM time step, following Alg. 1
// of Rettinger & Ruede (arXiv 1711.00336, Sec. 3.3).
//
// Layout: cell fields are structure-of-arrays [ncomp][nc] with x fastest, so
// a 64-lane wavefront touches 64 consecutive cells of one component. PDFs
// are stored as deviations f_q - w_q (rho_0 = 1) in float or double.
// Particles are SoA [3][cap] doubles kept sorted by (cell, insertion index).
// Particle -> cell transfers are gathers: every cell sums the particles of
// its 3x3x3 neighbouring 1-cell bins (contiguous slot ranges), so the result
// is deterministic and needs no floating-point atomics.
#include "lbdem_internal.h"

#include <mutex>

#include <cmath>

namespace lbdem {

// ---------------------------------------------------------------------------
// D3Q19 velocity set: 0 rest; 1..6 +x,-x,+y,-y,+z,-z; 7..18 face diagonals
// (1,1,0),(-1,-1,0),(1,-1,0),(-1,1,0),(1,0,1),(-1,0,-1),(1,0,-1),(-1,0,1),
// (0,1,1),(0,-1,-1),(0,1,-1),(0,-1,1). Weights 1/3, 1/18, 1/36.
// Written as constexpr selectors so that unrolled loops fold to immediates.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int CX(int q)
{
    return (q == 1 || q == 7 || q == 9 || q == 11 || q == 13) ? 1
         : (q == 2 || q == 8 || q == 10 || q == 12 || q == 14) ? -1 : 0;
}
__host__ __device__ constexpr int CY(int q)
{
    return (q == 3 || q == 7 || q == 10 || q == 15 || q == 17) ? 1
         : (q == 4 || q == 8 || q == 9 || q == 16 || q == 18) ? -1 : 0;
}
__host__ __device__ constexpr int CZ(int q)
{
    return (q == 5 || q == 11 || q == 14 || q == 15 || q == 18) ? 1
         : (q == 6 || q == 12 || q == 13 || q == 16 || q == 17) ? -1 : 0;
}
__host__ __device__ constexpr int CC(int q, int a) { return a == 0 ? CX(q) : a == 1 ? CY(q) : CZ(q); }
__host__ __device__ constexpr double WQ(int q) { return q == 0 ? 1.0 / 3.0 : q <= 6 ? 1.0 / 18.0 : 1.0 / 36.0; }
__host__ __device__ constexpr int OPP(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2. Remap the hardware block id so that every XCD walks one contiguous
// range of logical blocks (a slab of cells or a run of cell-sorted
// particles): stencil neighbours then hit the same L2. A bijection on
// [0, nblocks) for any dispatch order, so only performance depends on it.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nb)
{
    const uint32_t per = nb >> 3, rem = nb & 7u, x = b & 7u, idx = b >> 3;
    return x < rem ? x * (per + 1) + idx : rem * (per + 1) + (x - rem) * per + idx;
}

__device__ __forceinline__ int64_t gidx(int64_t per_block = kBlock)
{
    return (int64_t)xcd_remap(blockIdx.x, gridDim.x) * per_block + threadIdx.x;
}

// wrap a coordinate that is at most one period outside [0, n)
__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ uint32_t fdiv(uint32_t c, uint32_t m, uint32_t s)
{
    return (__umulhi(c, m) + c) >> s;
}

__device__ __forceinline__ void cell_coords(const Geo &g, int64_t c64, int &i, int &j, int &k)
{
    const uint32_t c = (uint32_t)c64;
    const uint32_t kk = fdiv(c, g.mxy, g.sxy);
    const uint32_t rem = c - kk * (uint32_t)(g.n[0] * g.n[1]);
    const uint32_t jj = fdiv(rem, g.mx, g.sx);
    i = (int)(rem - jj * (uint32_t)g.n[0]);
    j = (int)jj;
    k = (int)kk;
}

__device__ __forceinline__ int64_t cidx(const Geo &g, int i, int j, int k)
{
    return (int64_t)i + (int64_t)g.n[0] * ((int64_t)j + (int64_t)g.n[1] * k);
}

// ---------------------------------------------------------------------------
// Roma et al. three-point kernel (Sec. 3.1.2, Eq. filter_def), applied per
// axis; the 3-D weight is the product over axes. Walled axes drop cells
// outside the domain and renormalise the rest to unit sum.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double roma(double r)
{
    r = fabs(r);
    if (r < 0.5) return (1.0 + sqrt(1.0 - 3.0 * r * r)) / 3.0;
    if (r < 1.5) return (5.0 - 3.0 * r - sqrt(1.0 - 3.0 * (1.0 - r) * (1.0 - r))) / 6.0;
    return 0.0;
}

// per-axis kernel weights of a particle at xp: cells b-1, b, b+1 with
// b = floor(xp); out-of-domain cells on walled axes get weight 0 and the
// others are divided by their sum.
__device__ __forceinline__ void axis_weights(double xp, int n, int per, int &b, double w[3])
{
    b = (int)floor(xp);
    if (per) b = b < 0 ? 0 : (b >= n ? n - 1 : b);
    double sum = 0.0;
#pragma unroll
    for (int o = -1; o <= 1; ++o) {
        const int i = b + o;
        const double wo = roma((double)i + 0.5 - xp);
        if (per || (i >= 0 && i < n)) {
            w[o + 1] = wo;
            sum += wo;
        } else {
            w[o + 1] = 0.0;
        }
    }
    if (!per) {
#pragma unroll
        for (int o = 0; o < 3; ++o) w[o] /= sum;
    }
}

// cell coordinate of stencil offset o (clamped on walled axes, where the
// weight of an out-of-domain offset is zero)
__device__ __forceinline__ int stencil_coord(int b, int o, int n, int per)
{
    int i = b + o;
    if (per) return wrap1(i, n);
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// distinct wrapped coordinates c-r..c+r on one axis (walled: in range only)
__device__ __forceinline__ int axis_range(int c, int r, int n, int per, int *out, int cap)
{
    int m = 0;
    if (per) {
        if (2 * r + 1 >= n) {
            for (int i = 0; i < n && m < cap; ++i) out[m++] = i;
        } else {
            for (int o = -r; o <= r; ++o) out[m++] = wrap1(c + o, n);
        }
    } else {
        for (int o = -r; o <= r; ++o) {
            const int i = c + o;
            if (i >= 0 && i < n) out[m++] = i;
        }
    }
    return m;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ int64_t particle_cell(const Geo &g, double x, double y, double z)
{
    const int i = clampi((int)floor(x), 0, g.n[0] - 1);
    const int j = clampi((int)floor(y), 0, g.n[1] - 1);
    const int k = clampi((int)floor(z), 0, g.n[2] - 1);
    return cidx(g, i, j, k);
}

__device__ __forceinline__ double sphere_volume(double d) { return M_PI * d * d * d / 6.0; }

// 4-vector cell fields ([nc][4], components x, y, z, 0): one 16- or 32-byte
// access per cell instead of three scattered ones
__device__ __forceinline__ void store_vec4(float *p, float a, float b, float c)
{
    *reinterpret_cast<float4 *>(p) = make_float4(a, b, c, 0.0f);
}
__device__ __forceinline__ void store_vec4(double *p, double a, double b, double c)
{
    reinterpret_cast<double2 *>(p)[0] = make_double2(a, b);
    reinterpret_cast<double2 *>(p)[1] = make_double2(c, 0.0);
}
__device__ __forceinline__ void load_vec4(const float *p, float v[3])
{
    const float4 t = *reinterpret_cast<const float4 *>(p);
    v[0] = t.x;
    v[1] = t.y;
    v[2] = t.z;
}
__device__ __forceinline__ void load_vec4(const double *p, double v[3])
{
    const double2 a = reinterpret_cast<const double2 *>(p)[0], b = reinterpret_cast<const double2 *>(p)[1];
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
}

// ---------------------------------------------------------------------------
// a1: moments of the post-stream PDFs (Eq. MacVel): rho - 1 = sum df,
// j = sum c df (exact with deviations since sum_q w_q c_q = 0).
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kBlock) void k_moments(Desc D, Cells<R> C)
{
    const int64_t nc = D.g.nc;
    const int64_t c = gidx();
    if (c >= nc) return;
    R r = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        const R f = C.df_src[q * nc + c];
        r += f;
        if (CX(q) > 0) jx += f; else if (CX(q) < 0) jx -= f;
        if (CY(q) > 0) jy += f; else if (CY(q) < 0) jy -= f;
        if (CZ(q) > 0) jz += f; else if (CZ(q) < 0) jz -= f;
    }
    C.drho[c] = r;
    C.j[c] = jx;
    C.j[nc + c] = jy;
    C.j[2 * nc + c] = jz;
    // fluid-phase velocity with the body force only (Eq. MacVel, u_f = u_bar/eps_f);
    // with lift also the first subcycle's u_f, from which its curl is taken
    const double e = 1.0 - (double)C.epsp[c];
    const double rho = 1.0 + (double)r;
    const R u0 = (R)(((double)jx + 0.5 * e * D.p.fb[0]) / (rho * e));
    const R u1 = (R)(((double)jy + 0.5 * e * D.p.fb[1]) / (rho * e));
    const R u2 = (R)(((double)jz + 0.5 * e * D.p.fb[2]) / (rho * e));
    C.un[c] = u0;
    C.un[nc + c] = u1;
    C.un[2 * nc + c] = u2;
    if (D.p.use_lift) {
        C.uf[c] = u0;
        C.uf[nc + c] = u1;
        C.uf[2 * nc + c] = u2;
    }
}

// Neighbours x + c_q with the wall ghost rule: the mirrored in-domain cell;
// a velocity flips sign once per mirrored axis (no-slip at the half-way
// plane), a scalar keeps its value. Resolved once per cell and axis: o[a][d+1]
// is the flat-index term of coordinate (i_a + d) (times 1, nx or nx*ny;
// 32-bit, since a domain has fewer than 2^31 cells) and s[a][d+1] the sign a
// velocity takes there.
struct Nbh {
    int o[3][3];
    double s[3][3];
};

__device__ __forceinline__ void neighbourhood(const Geo &g, int i, int j, int k, Nbh &h)
{
    const int c[3] = {i, j, k};
    const int stride[3] = {1, g.n[0], g.n[0] * g.n[1]};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int d = -1; d <= 1; ++d) {
            int t = c[a] + d;
            double sg = 1.0;
            if (t < 0 || t >= g.n[a]) {
                if (g.per[a]) t = wrap1(t, g.n[a]);
                else {
                    t = c[a];
                    sg = -1.0;
                }
            }
            h.o[a][d + 1] = t * stride[a];
            h.s[a][d + 1] = sg;
        }
}

// flat index and velocity sign of neighbour x + c_q (q a compile-time constant
// in unrolled loops, so the table lookups are register selects)
__device__ __forceinline__ int ghost(const Nbh &h, int q, double &sign)
{
    sign = h.s[0][CX(q) + 1] * h.s[1][CY(q) + 1] * h.s[2][CZ(q) + 1];
    return h.o[0][CX(q) + 1] + h.o[1][CY(q) + 1] + h.o[2][CZ(q) + 1];
}

// ---------------------------------------------------------------------------
// a2/a3: per-step cell fields (Alg. 1, the step before the subcycle loop,
// which keeps the material derivative fixed for the whole LBM step):
//   u_f^n = (j + eps_f f_b / 2) / (rho eps_f)      (Eq. MacVel, u_f = u_bar/eps_f)
//   Du_f/Dt = (u_f^n - u_prev) + (u_f^n . grad_L) u_f^n (0 time part at step 0)
//   grad P = (1/c_s^2) sum_q w_q c_q P(x+c_q) = sum_q w_q c_q (rho-1)(x+c_q)
// with the lattice gradient of Sec. 3.2.3. Also resets f_acc.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kBlock) void k_cellfields(Desc D, Cells<R> C)
{
    const int64_t nc = D.g.nc;
    const int64_t c = gidx();
    if (c >= nc) return;
    int i, j, k;
    cell_coords(D.g, c, i, j, k);
    Nbh h;
    neighbourhood(D.g, i, j, k, h);
    double G[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    double gp[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        double sg;
        const int64_t nb = ghost(h, q, sg);
        const double u0 = (double)C.un[nb];
        const double u1 = (double)C.un[nc + nb];
        const double u2 = (double)C.un[2 * nc + nb];
        const double dr = (double)C.drho[nb];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (CC(q, a) == 0) continue;
            const double wc = CC(q, a) > 0 ? WQ(q) : -WQ(q);
            G[a][0] += wc * (sg * u0);
            G[a][1] += wc * (sg * u1);
            G[a][2] += wc * (sg * u2);
            gp[a] += wc * dr;
        }
    }
    double un[3];
    un[0] = (double)C.un[c];
    un[1] = (double)C.un[nc + c];
    un[2] = (double)C.un[2 * nc + c];
    const bool have_prev = *D.stepc > 0;
    R du[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        double conv = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) conv += un[a] * (3.0 * G[a][b]);
        const double dtu = have_prev ? (un[b] - (double)C.uprev[b * nc + c]) : 0.0;
        du[b] = (R)(dtu + conv);
        C.gradp[b * nc + c] = (R)gp[b];
        C.uprev[b * nc + c] = (R)un[b];
        C.facc[b * nc + c] = (R)0;
    }
    store_vec4(C.dudt + 4 * c, du[0], du[1], du[2]);
}

// ---------------------------------------------------------------------------
// Lift only, at every subcycle start (Alg. 1, the first step inside the
// subcycle loop, which also needs u_f; grad P depends on rho alone and comes
// from the per-step pass): the lattice curl of Sec. 3.2.3,
//   curl u_f(x) = (1/c_s^2) sum_q w_q c_q x u_f(x + c_q),
// of the subcycle-start u_f = (j + eps_f f_b / 2) / (rho eps_f) that the
// moments pass (first subcycle) or the volume-fraction gather (later ones)
// leaves in uf; neighbours beyond a wall by the velocity ghost rule above.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kBlock) void k_curl(Desc D, Cells<R> C)
{
    const int64_t nc = D.g.nc;
    const int64_t c = gidx();
    if (c >= nc) return;
    int i, j, k;
    cell_coords(D.g, c, i, j, k);
    Nbh h;
    neighbourhood(D.g, i, j, k, h);
    double s[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 1; q < 19; ++q) {
        double sg;
        const int64_t nb = ghost(h, q, sg);
        const double u0 = sg * (double)C.uf[nb], u1 = sg * (double)C.uf[nc + nb], u2 = sg * (double)C.uf[2 * nc + nb];
        s[0] += WQ(q) * (CY(q) * u2 - CZ(q) * u1);
        s[1] += WQ(q) * (CZ(q) * u0 - CX(q) * u2);
        s[2] += WQ(q) * (CX(q) * u1 - CY(q) * u0);
    }
    store_vec4(C.curl + 4 * c, (R)(3.0 * s[0]), (R)(3.0 * s[1]), (R)(3.0 * s[2]));
}

// ---------------------------------------------------------------------------
// a4: added mass (Table 1): F_am = C_am rho_f V (Du_f/Dt|_p - du_p/dt), the
// fluid derivative interpolated with Eq. interpolation. Also records the
// subcycle-start velocity and position.
// ---------------------------------------------------------------------------
struct Stencil {
    int b[3];
    double w[3][3];
};

// stored kernel weight u (= 3*axis + o+1) of slot p, in the storage precision
template <typename R> __device__ __forceinline__ R stencil_weight(const Parts &P, int u, int64_t p);
template <> __device__ __forceinline__ float stencil_weight<float>(const Parts &P, int u, int64_t p)
{
    return P.swf[u * P.cap + p];
}
template <> __device__ __forceinline__ double stencil_weight<double>(const Parts &P, int u, int64_t p)
{
    return P.sw[u * P.cap + p];
}

template <typename R> __device__ __forceinline__ void load_stencil(const Parts &P, int64_t i, Stencil &st)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        st.b[a] = P.sb[a * P.cap + i];
#pragma unroll
        for (int o = 0; o < 3; ++o) st.w[a][o] = (double)stencil_weight<R>(P, 3 * a + o, i);
    }
}

// st.w[a][o] for a runtime o without indexing a register array
__device__ __forceinline__ double sel3(const double w[3], int o) { return o == 0 ? w[0] : (o == 1 ? w[1] : w[2]); }

// F_am = C_am rho_f V (Du/Dt|p - a_p) (Table 1) of slot i from the particle's
// diameter, du_p/dt, velocity and position; records the subcycle-start
// velocity and position
template <typename R>
__device__ __forceinline__ void am_store(const Desc &D, int64_t i, const R Du[3], double d, const double a[3],
                                         const double u[3], const double x[3])
{
    const Parts &P = D.pt;
    const int64_t cap = P.cap;
    const R V = (R)sphere_volume(d);
    const R cam = (R)(D.p.c_am * D.p.rho_f);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const R F = D.p.use_am ? cam * V * (Du[b] - (R)a[b]) : (R)0;
        P.Fam[b * cap + i] = (double)F;
        P.ustart[b * cap + i] = u[b];
        P.xstart[b * cap + i] = x[b];
    }
}

// the same for the particle in slot i (subcycle start state)
template <typename R> __device__ __forceinline__ void am_force(const Desc &D, int64_t i, const R Du[3])
{
    const Parts &P = D.pt;
    const int64_t cap = P.cap;
    double a[3], u[3], x[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        a[b] = P.a[b * cap + i];
        u[b] = P.u[b * cap + i];
        x[b] = P.x[b * cap + i];
    }
    am_store<R>(D, i, Du, P.d[i], a, u, x);
}

// Du_f/Dt|p = sum of the 27 stencil cells' Du_f/Dt with the stored weights
// (Eq. interpolation), summed in R in the order (z, y, x)
template <typename R>
__device__ __forceinline__ void interp_dudt(const Desc &D, const Cells<R> &C, const Stencil &st, R Du[3])
{
#pragma unroll 1
    for (int oz = 0; oz < 3; ++oz) {
        const int cz = stencil_coord(st.b[2], oz - 1, D.g.n[2], D.g.per[2]);
#pragma unroll
        for (int oy = 0; oy < 3; ++oy) {
            const int cy = stencil_coord(st.b[1], oy - 1, D.g.n[1], D.g.per[1]);
#pragma unroll
            for (int ox = 0; ox < 3; ++ox) {
                const int cx = stencil_coord(st.b[0], ox - 1, D.g.n[0], D.g.per[0]);
                const int64_t cell = cidx(D.g, cx, cy, cz);
                const R w = (R)(st.w[0][ox] * st.w[1][oy] * sel3(st.w[2], oz));
                R v[3];
                load_vec4(C.dudt + 4 * cell, v);
#pragma unroll
                for (int b = 0; b < 3; ++b) Du[b] += w * v[b];
            }
        }
    }
}

// F_l = 1.61 d^2 sqrt(mu rho_f / |w_f|) ((u_f|p - u_p) x w_f) (Table 1, lift),
// w_f = (curl u_f)|p; zero where w_f = 0 (the formula's limit). u_p and u_f
// are those of the subcycle start.
template <typename R> __device__ __forceinline__ void lift_force(const Desc &D, int64_t i, const R uf[3], const R om[3])
{
    const Parts &P = D.pt;
    const int64_t cap = P.cap;
    const R on = sqrt(om[0] * om[0] + om[1] * om[1] + om[2] * om[2]);
    R F[3] = {(R)0, (R)0, (R)0};
    if (on > (R)0) {
        R w[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) w[b] = uf[b] - (R)P.u[b * cap + i];
        const R d = (R)P.d[i];
        const R s = (R)1.61 * d * d * sqrt((R)D.p.mu * (R)D.p.rho_f / on);
        F[0] = s * (w[1] * om[2] - w[2] * om[1]);
        F[1] = s * (w[2] * om[0] - w[0] * om[2]);
        F[2] = s * (w[0] * om[1] - w[1] * om[0]);
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) P.Fl[b * cap + i] = (double)F[b];
}

// interpolation sums and the added-mass force (and with LIFT the lift from
// the interpolated u_f and curl u_f) in the cell precision R (FP32 in the
// FP32-deviation form); the forces are stored FP64
template <typename R, bool LIFT>
__global__ __launch_bounds__(kBlock) void k_part_am(Desc D, Cells<R> C)
{
    const int64_t i = gidx();
    const Parts &P = D.pt;
    if (i >= P.np) return;
    const int64_t nc = D.g.nc;
    Stencil st;
    load_stencil<R>(P, i, st);
    R Du[3] = {(R)0, (R)0, (R)0};
    R U[3] = {(R)0, (R)0, (R)0}, Om[3] = {(R)0, (R)0, (R)0};
    if (!LIFT) {
        interp_dudt<R>(D, C, st, Du);
        am_force<R>(D, i, Du);
        return;
    }
#pragma unroll 1
    for (int oz = 0; oz < 3; ++oz) {
        const int cz = stencil_coord(st.b[2], oz - 1, D.g.n[2], D.g.per[2]);
#pragma unroll
        for (int oy = 0; oy < 3; ++oy) {
            const int cy = stencil_coord(st.b[1], oy - 1, D.g.n[1], D.g.per[1]);
#pragma unroll
            for (int ox = 0; ox < 3; ++ox) {
                const int cx = stencil_coord(st.b[0], ox - 1, D.g.n[0], D.g.per[0]);
                const int64_t cell = cidx(D.g, cx, cy, cz);
                const R w = (R)(st.w[0][ox] * st.w[1][oy] * sel3(st.w[2], oz));
                R v[3];
                load_vec4(C.dudt + 4 * cell, v);
#pragma unroll
                for (int b = 0; b < 3; ++b) Du[b] += w * v[b];
                if (LIFT) {
                    R o[3];
                    load_vec4(C.curl + 4 * cell, o);
#pragma unroll
                    for (int b = 0; b < 3; ++b) {
                        U[b] += w * C.uf[b * nc + cell];
                        Om[b] += w * o[b];
                    }
                }
            }
        }
    }
    am_force<R>(D, i, Du);
    if (LIFT) lift_force<R>(D, i, U, Om);
}

// ---------------------------------------------------------------------------
// Gather of a particle quantity to one cell (Eq. distribution_filter with
// D = I): s = sum_p D(x, x_p) v_p over the particles of the 3x3x3
// neighbouring bins. Slots are sorted by cell, so each x-row of three bins is
// one contiguous slot range.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ double stencil_w(const Parts &P, int64_t p, int axis, int ic, int n, int per)
{
    const int b = P.sb[axis * P.cap + p];
    int o = ic - b;
    if (per) {
        if (n < 3) {  // several stencil offsets land on the same cell
            double w = 0.0;
#pragma unroll
            for (int t = -1; t <= 1; ++t)
                if (wrap1(b + t, n) == ic) w += (double)stencil_weight<R>(P, 3 * axis + t + 1, p);
            return w;
        }
        o = o > 1 ? o - n : (o < -1 ? o + n : o);
    }
    return (o >= -1 && o <= 1) ? (double)stencil_weight<R>(P, 3 * axis + o + 1, p) : 0.0;
}

// weights and values in the storage precision R, products accumulated in
// FP64 (the same arithmetic as the LDS tiles, so all variants agree)
template <typename R, int NV, typename F>
__device__ __forceinline__ void gather_range(const Desc &D, int i, int j, int k, int p0, int p1, const F &val,
                                             double *s)
{
    for (int p = p0; p < p1; ++p) {
        const R wx = (R)stencil_w<R>(D.pt, p, 0, i, D.g.n[0], D.g.per[0]);
        const R wy = (R)stencil_w<R>(D.pt, p, 1, j, D.g.n[1], D.g.per[1]);
        const R wz = (R)stencil_w<R>(D.pt, p, 2, k, D.g.n[2], D.g.per[2]);
        const R w = wx * wy * wz;
        if (w == (R)0) continue;
        double v[NV];
        val(p, v);
#pragma unroll
        for (int q = 0; q < NV; ++q) s[q] += (double)w * (double)(R)v[q];
    }
}

template <typename R, int NV, typename F>
__device__ __forceinline__ void gather_cell(const Desc &D, int i, int j, int k, const F &val, double *s)
{
    int cx[3], cy[3], cz[3];
    const int mx = axis_range(i, 1, D.g.n[0], D.g.per[0], cx, 3);
    const int my = axis_range(j, 1, D.g.n[1], D.g.per[1], cy, 3);
    const int mz = axis_range(k, 1, D.g.n[2], D.g.per[2], cz, 3);
    // one contiguous x-run of bins when the row does not wrap
    const bool run = mx == 3 && cx[0] + 2 == cx[2];
#pragma unroll
    for (int t = 0; t < NV; ++t) s[t] = 0.0;
    for (int a = 0; a < mz; ++a)
        for (int b = 0; b < my; ++b) {
            if (run) {
                const int64_t b0 = cidx(D.g, cx[0], cy[b], cz[a]);
                gather_range<R, NV>(D, i, j, k, D.b.start[b0], D.b.start[b0 + 3], val, s);
            } else {
                for (int c = 0; c < mx; ++c) {
                    const int64_t bin = cidx(D.g, cx[c], cy[b], cz[a]);
                    gather_range<R, NV>(D, i, j, k, D.b.start[bin], D.b.start[bin + 1], val, s);
                }
            }
        }
}

// ---------------------------------------------------------------------------
// LDS-tiled gather. A workgroup owns a TX x TY x (TZ*CZ) tile of cells, each
// thread CZ consecutive cells along z. It counts the particles of the tile's
// halo bins (the tile widened by one cell, wrapped on periodic axes), lists
// their slots in LDS (a bin's particles are one contiguous slot range, listed
// by the thread that owns the bin), stages their stencils and values into
// LDS one entry per thread (independent, coalesced loads), and then every cell
// sums the particles of its own 3x3x3 bins from LDS, in the order
// (dz, dy, dx, slot) whatever the tile shape. Tiles whose halo holds more
// than KMAX particles fall back to the per-cell global gather.
//   MODE_AM : fam  = -sum_p D (F_am + F_l)            (Eq. forces_pf, added mass, lift)
//   MODE_FD : facc += (eps_f f_b + fam - sum_p D F_d) / n_int   (mean f_ext)
//   MODE_EPS: epsp = sum_p D V_p                      (Eq. fluid_volume_fraction)
//   MODE_EPS_AM: both of the new positions: the volume fraction at the end of
//            one subcycle and the added-mass spreading of the next one
//   MODE_EPS_UF: the volume fraction and, for the lift's curl, the next
//            subcycle's starting u_f = (j + eps_f f_b/2) / (rho eps_f)
// MODE_AM and MODE_EPS_AM also store the re-evaluated fluid-phase velocity
// u_f = (j + (eps_f f_b + fam)/2) / (rho eps_f) (Sec. 3.2.3, Alg. 1).
// ---------------------------------------------------------------------------
enum { MODE_AM = 0, MODE_FD = 1, MODE_EPS = 2, MODE_EPS_AM = 3, MODE_EPS_UF = 4 };

template <int MODE> struct GatherNV {
    static constexpr int v = (MODE == MODE_EPS || MODE == MODE_EPS_UF) ? 1 : (MODE == MODE_EPS_AM ? 4 : 3);
};

template <int MODE>
__device__ __forceinline__ void gather_value(const Parts &P, int p, double *v)
{
    if (MODE == MODE_EPS || MODE == MODE_EPS_UF) {
        v[0] = sphere_volume(P.d[p]);
    } else if (MODE == MODE_EPS_AM) {
        v[0] = sphere_volume(P.d[p]);
        v[1] = P.Fam[p];
        v[2] = P.Fam[P.cap + p];
        v[3] = P.Fam[2 * P.cap + p];
    } else {
        const double *F = MODE == MODE_AM ? P.Fam : P.Fd;
        v[0] = F[p];
        v[1] = F[P.cap + p];
        v[2] = F[2 * P.cap + p];
        if (MODE == MODE_AM && P.Fl) {  // lift, spread together with the added mass
            v[0] += P.Fl[p];
            v[1] += P.Fl[P.cap + p];
            v[2] += P.Fl[2 * P.cap + p];
        }
    }
}

template <typename R>
__device__ __forceinline__ void store_fam_uf(const Desc &D, const Cells<R> &C, int64_t c, double e, const double *sam)
{
    const int64_t nc = D.g.nc;
    const double rho = 1.0 + (double)C.drho[c];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const R fam = (R)(-sam[b]);
        C.fam[b * nc + c] = fam;
        const double fext = e * D.p.fb[b] + (double)fam;
        C.uf[b * nc + c] = (R)(((double)C.j[b * nc + c] + 0.5 * fext) / (rho * e));
    }
}

template <typename R, int MODE>
__device__ __forceinline__ void gather_store(const Desc &D, const Cells<R> &C, int64_t c, const double *s)
{
    const int64_t nc = D.g.nc;
    if (MODE == MODE_AM) {
        store_fam_uf<R>(D, C, c, 1.0 - (double)C.epsp[c], s);
    } else if (MODE == MODE_EPS_AM) {
        const double e = 1.0 - s[0];
        if (!(e > 0.0) || !isfinite(e)) atomicOr(D.flags, FLAG_EPS);
        C.epsp[c] = (R)s[0];
        store_fam_uf<R>(D, C, c, 1.0 - (double)(R)s[0], s + 1);
    } else if (MODE == MODE_FD) {
        const double e = 1.0 - (double)C.epsp[c];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double fext = e * D.p.fb[b] + (double)C.fam[b * nc + c] - s[b];
            C.facc[b * nc + c] = (R)((double)C.facc[b * nc + c] + fext * D.p.dt_int);
        }
    } else {
        const double e = 1.0 - s[0];
        if (!(e > 0.0) || !isfinite(e)) atomicOr(D.flags, FLAG_EPS);
        C.epsp[c] = (R)s[0];
        if (MODE == MODE_EPS_UF) {
            const double ef = 1.0 - (double)(R)s[0];
            const double rho = 1.0 + (double)C.drho[c];
#pragma unroll
            for (int b = 0; b < 3; ++b)
                C.uf[b * nc + c] = (R)(((double)C.j[b * nc + c] + 0.5 * ef * D.p.fb[b]) / (rho * ef));
        }
    }
}

template <typename R, int MODE, int TX, int TY, int TZ, int CZ, int KMAX>
__global__ __launch_bounds__(TX *TY *TZ) void k_gather_tile(Desc D, Cells<R> C)
{
    constexpr int NT = TX * TY * TZ, HX = TX + 2, HY = TY + 2, HZ = TZ * CZ + 2, NHB = HX * HY * HZ;
    constexpr int NV = GatherNV<MODE>::v;
    constexpr int PER = (NHB + NT - 1) / NT;
    constexpr int NW = NT / 64;
    static_assert(NT % 64 == 0, "whole wavefronts");
    __shared__ int hoff[NHB + 1];
    __shared__ int wsum[NW];
    // staged weights and values in the storage precision R (halves LDS in the
    // FP32 form); products are accumulated in FP64
    __shared__ R sw_l[9][KMAX];
    __shared__ R sv_l[NV][KMAX];
    __shared__ int sslot[KMAX];  // particle slot of each staged entry

    const int tid = threadIdx.x;
    const int n0 = D.g.n[0], n1 = D.g.n[1], n2 = D.g.n[2];
    const uint32_t lin = xcd_remap(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                                   gridDim.x * gridDim.y * gridDim.z);
    const int bx = (int)(lin % gridDim.x), by = (int)((lin / gridDim.x) % gridDim.y),
              bz = (int)(lin / (gridDim.x * gridDim.y));
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ * CZ;
    // halo bins beyond the last cell of a partial tile (+1) are not needed
    const int lx = min(x0 + TX, n0) - x0 + 1, ly = min(y0 + TY, n1) - y0 + 1,
              lz = min(z0 + TZ * CZ, n2) - z0 + 1;

    // each thread owns PER consecutive halo bins
    int src[PER], cnt[PER];
    int sum = 0;
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int hb = tid * PER + t;
        src[t] = 0;
        cnt[t] = 0;
        if (hb < NHB) {
            const int hx = hb % HX, hy = (hb / HX) % HY, hz = hb / (HX * HY);
            int g[3] = {x0 - 1 + hx, y0 - 1 + hy, z0 - 1 + hz};
            bool ok = hx <= lx && hy <= ly && hz <= lz;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (g[a] < 0 || g[a] >= D.g.n[a]) {
                    if (D.g.per[a]) g[a] = wrap1(g[a], D.g.n[a]);
                    else ok = false;
                }
            }
            if (ok) {
                const int64_t bin = cidx(D.g, g[0], g[1], g[2]);
                src[t] = D.b.start[bin];
                cnt[t] = D.b.start[bin + 1] - src[t];
            }
        }
        sum += cnt[t];
    }
    // exclusive scan of the per-thread counts: wavefront shuffles, then the
    // wavefront totals through LDS (one barrier)
    const int lane = tid & 63, wv = tid >> 6;
    int incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int run = incl - sum, K = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const int ws = wsum[w];
        if (w < wv) run += ws;
        K += ws;
    }
    // offsets of the halo bins and the particle slot of every staged entry
    // (written by the thread that owns the bin: LDS stores only) ...
    const Parts &P = D.pt;
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int hb = tid * PER + t;
        if (hb < NHB) hoff[hb] = run;
        if (K <= KMAX)
            for (int q = 0; q < cnt[t]; ++q) sslot[run + q] = src[t] + q;
        run += cnt[t];
    }
    if (tid == NT - 1) hoff[NHB] = K;
    __syncthreads();
    // ... then the staging of weights and values, one entry per thread, so
    // that a wavefront's loads are independent (same entries, same order)
    if (K <= KMAX) {
        for (int kk = tid; kk < K; kk += NT) {
            const int p = sslot[kk];
#pragma unroll
            for (int u = 0; u < 9; ++u) sw_l[u][kk] = stencil_weight<R>(P, u, p);
            double v[NV];
            gather_value<MODE>(P, p, v);
#pragma unroll
            for (int u = 0; u < NV; ++u) sv_l[u][kk] = (R)v[u];
        }
        __syncthreads();
    }

    const int tx = tid % TX, ty = (tid / TX) % TY, tz = tid / (TX * TY);
    const int i = x0 + tx, j = y0 + ty, kb = z0 + tz * CZ;
    if (i >= n0 || j >= n1) return;
    double s[CZ][NV];

    if (K > KMAX) {  // crowded tile: per-cell gather from global memory
#pragma unroll
        for (int c = 0; c < CZ; ++c) {
            if (kb + c >= n2) break;
            gather_cell<R, NV>(D, i, j, kb + c, [&](int p, double *v) { gather_value<MODE>(D.pt, p, v); }, s[c]);
            gather_store<R, MODE>(D, C, cidx(D.g, i, j, kb + c), s[c]);
        }
        return;
    }

#pragma unroll
    for (int c = 0; c < CZ; ++c)
#pragma unroll
        for (int t = 0; t < NV; ++t) s[c][t] = 0.0;
    // The bin of a staged particle fixes its stencil offset relative to a
    // cell: a particle in bin (i-1+dx, j-1+dy, k-1+dz) sees the cell at offset
    // (1-dx, 1-dy, 1-dz), i.e. weight slots 2-dx, 2-dy, 2-dz of its axes.
    // Halo row r (z = kb - 1 + r) feeds the thread's cells c with dz = r - c.
#pragma unroll
    for (int r = 0; r < CZ + 2; ++r)
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const int hb0 = ((tz * CZ + r) * HY + (ty + dy)) * HX + tx;
            const int k0 = hoff[hb0], k1 = hoff[hb0 + 1], k2 = hoff[hb0 + 2], k3 = hoff[hb0 + 3];
            for (int kk = k0; kk < k3; ++kk) {
                const int sx = kk < k1 ? 2 : (kk < k2 ? 1 : 0);
                const R wxy = sw_l[sx][kk] * sw_l[3 + 2 - dy][kk];
                R v[NV];
#pragma unroll
                for (int t = 0; t < NV; ++t) v[t] = sv_l[t][kk];
#pragma unroll
                for (int c = 0; c < CZ; ++c) {
                    const int dz = r - c;
                    if (dz < 0 || dz > 2) continue;
                    const R w = wxy * sw_l[6 + 2 - dz][kk];
#pragma unroll
                    for (int t = 0; t < NV; ++t) s[c][t] += (double)w * (double)v[t];
                }
            }
        }
#pragma unroll
    for (int c = 0; c < CZ; ++c)
        if (kb + c < n2) gather_store<R, MODE>(D, C, cidx(D.g, i, j, kb + c), s[c]);
}

// per-cell global gather (thin periodic axes, where a cell's neighbour bins coincide)
template <typename R, int MODE>
__global__ __launch_bounds__(kBlock) void k_gather_cells(Desc D, Cells<R> C)
{
    const int64_t nc = D.g.nc;
    const int64_t c = gidx();
    if (c >= nc) return;
    int i, j, k;
    cell_coords(D.g, c, i, j, k);
    constexpr int NV = GatherNV<MODE>::v;
    double s[NV];
    gather_cell<R, NV>(D, i, j, k, [&](int p, double *v) { gather_value<MODE>(D.pt, p, v); }, s);
    gather_store<R, MODE>(D, C, c, s);
}

// ---------------------------------------------------------------------------
// a6: pressure-gradient force, drag, gravity + buoyancy (Table 1, Sec. 3.1.2)
// with u_f re-evaluated from f_ext = eps_f f_b + f_am (Sec. 3.2.3 stability
// measures; Alg. 1, the u_f update between the two particle loops).
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ T drag_factor(T Re, T ep)
{
    const T e1 = (T)1 - ep;
    const T cd0 = (T)1 + (T)0.15 * (Re > (T)0 ? pow(Re, (T)0.687) : (T)0);
    const T A = (T)5.81 * ep / (e1 * e1 * e1) + (T)0.48 * (ep > (T)0 ? cbrt(ep) : (T)0) / (e1 * e1 * e1 * e1);
    const T B = ep * ep * ep * Re * ((T)0.95 + (T)0.61 * ep * ep * ep / (e1 * e1));
    const T cd = e1 * (cd0 / (e1 * e1 * e1) + A + B);
    return e1 * cd;
}

// F_pr = -V grad P|p, F_d (Tenneti closure as the paper prints it, Table 1),
// gravity and buoyancy; F_const for the DEM substeps
template <typename R>
__device__ __forceinline__ void drag_forces(const Desc &D, int64_t i, const R uf[3], const R gp[3], R ep, int record)
{
    const Parts &P = D.pt;
    const int64_t cap = P.cap;
    const double dd = P.d[i];
    const R d = (R)dd;
    const R V = (R)sphere_volume(dd);
    const R mu = (R)D.p.mu, rho_f = (R)D.p.rho_f;
    R wv[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) wv[b] = uf[b] - (R)P.u[b * cap + i];
    const R wn = sqrt(wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2]);
    const R Re = ((R)1 - ep) * rho_f * d * wn / mu;
    const R fac = (R)3 * (R)M_PI * d * mu * drag_factor(Re, ep);
    const R rp = (R)P.rho[i];
    const int pid = P.id[i];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const R Fpr = -V * gp[b];
        const R Fd = fac * wv[b];
        const R fgb = (rp - rho_f) * V * (R)D.p.g[b];
        const R Fam = (R)P.Fam[b * cap + i];
        const R Fl = P.Fl ? (R)P.Fl[b * cap + i] : (R)0;
        const R Fc = Fd + Fpr + Fam + Fl + fgb;
        P.Fd[b * cap + i] = (double)Fd;
        P.Fc[b * cap + i] = (double)Fc;
        if (record) {
            P.Fam_id[b * cap + pid] = (double)Fam;
            P.Fd_id[b * cap + pid] = (double)Fd;
            P.Fpr_id[b * cap + pid] = (double)Fpr;
            P.Fc_id[b * cap + pid] = (double)Fc;
            if (P.Fl_id) P.Fl_id[b * cap + pid] = (double)Fl;
        }
    }
}

// interpolation sums and the closures in the cell precision R (FP32 in the
// FP32-deviation form); the forces are stored FP64
template <typename R>
__global__ __launch_bounds__(kBlock) void k_part_drag(Desc D, Cells<R> C, int record)
{
    const int64_t i = gidx();
    const Parts &P = D.pt;
    if (i >= P.np) return;
    const int64_t nc = D.g.nc;
    Stencil st;
    load_stencil<R>(P, i, st);
    R uf[3] = {(R)0, (R)0, (R)0}, gp[3] = {(R)0, (R)0, (R)0}, ep = (R)0;
#pragma unroll 1
    for (int oz = 0; oz < 3; ++oz) {
        const int cz = stencil_coord(st.b[2], oz - 1, D.g.n[2], D.g.per[2]);
#pragma unroll
        for (int oy = 0; oy < 3; ++oy) {
            const int cy = stencil_coord(st.b[1], oy - 1, D.g.n[1], D.g.per[1]);
#pragma unroll
            for (int ox = 0; ox < 3; ++ox) {
                const int cx = stencil_coord(st.b[0], ox - 1, D.g.n[0], D.g.per[0]);
                const int64_t cell = cidx(D.g, cx, cy, cz);
                const R w = (R)(st.w[0][ox] * st.w[1][oy] * sel3(st.w[2], oz));
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    uf[b] += w * C.uf[b * nc + cell];
                    gp[b] += w * C.gradp[b * nc + cell];
                }
                ep += w * C.epsp[cell];
            }
        }
    }
    drag_forces<R>(D, i, uf, gp, ep, record);
}

// ---------------------------------------------------------------------------
// LDS-tiled particle pass (a6 drag/pressure/gravity, and a4's added mass
// with lift; without lift the added mass runs per particle). A workgroup owns the particles whose bins lie in a TX x TY x TZ tile of cells
// (one contiguous slot range per x-row of bins). It loads the cell fields of
// the tile widened by one cell (wrapped on periodic axes, clamped on walled
// ones, as the per-particle stencil does) into LDS with coalesced loads, and
// every particle interpolates from LDS. The arithmetic and its order are
// those of k_part_am / k_part_drag, so the results are bit-identical.
// ---------------------------------------------------------------------------
enum { PASS_AM = 0, PASS_DRAG = 1, PASS_AML = 2 };

template <typename R, int PASS, int TX, int TY, int TZ>
__global__ __launch_bounds__(256) void k_part_tile(Desc D, Cells<R> C, int record)
{
    constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2, NHC = HX * HY * HZ;
    // Du/Dt | u_f, grad P, eps_p | Du/Dt, u_f, curl u_f
    constexpr int NV = PASS == PASS_AM ? 3 : (PASS == PASS_DRAG ? 7 : 9);
    constexpr int NR = TY * TZ;
    static_assert(NR <= 64, "rows of one tile are scanned by one wavefront");
    __shared__ R cv[NV][NHC];
    __shared__ int rp[NR + 1], rsrc[NR];

    const int tid = threadIdx.x;
    const int n0 = D.g.n[0], n1 = D.g.n[1], n2 = D.g.n[2];
    const int64_t nc = D.g.nc;
    const uint32_t lin = xcd_remap(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z),
                                   gridDim.x * gridDim.y * gridDim.z);
    const int bx = (int)(lin % gridDim.x), by = (int)((lin / gridDim.x) % gridDim.y),
              bz = (int)(lin / (gridDim.x * gridDim.y));
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
    const int xe = min(x0 + TX, n0);
    const int lx = xe - x0 + 1, ly = min(y0 + TY, n1) - y0 + 1, lz = min(z0 + TZ, n2) - z0 + 1;

    // own particles: one slot range per row of bins
    if (tid < 64) {
        int cnt = 0, src = 0;
        if (tid < NR) {
            const int y = y0 + tid % TY, z = z0 + tid / TY;
            if (y < n1 && z < n2) {
                src = D.b.start[cidx(D.g, x0, y, z)];
                cnt = D.b.start[cidx(D.g, xe - 1, y, z) + 1] - src;
            }
            rsrc[tid] = src;
        }
        int incl = cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(incl, off, 64);
            if ((tid & 63) >= off) incl += y;
        }
        if (tid < NR) rp[tid] = incl - cnt;
        if (tid == NR - 1) rp[NR] = incl;
    }
    // halo cell fields
    for (int hc = tid; hc < NHC; hc += 256) {
        const int hx = hc % HX, hy = (hc / HX) % HY, hz = hc / (HX * HY);
        R v[NV];
        if (hx <= lx && hy <= ly && hz <= lz) {
            const int gx = stencil_coord(x0, hx - 1, n0, D.g.per[0]);
            const int gy = stencil_coord(y0, hy - 1, n1, D.g.per[1]);
            const int gz = stencil_coord(z0, hz - 1, n2, D.g.per[2]);
            const int64_t cell = cidx(D.g, gx, gy, gz);
            if (PASS == PASS_AM) {
                load_vec4(C.dudt + 4 * cell, v);
            } else if (PASS == PASS_AML) {
                load_vec4(C.dudt + 4 * cell, v);
#pragma unroll
                for (int b = 0; b < 3; ++b) v[3 + b] = C.uf[b * nc + cell];
                load_vec4(C.curl + 4 * cell, v + 6);
            } else {
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    v[b] = C.uf[b * nc + cell];
                    v[3 + b] = C.gradp[b * nc + cell];
                }
                v[6] = C.epsp[cell];
            }
        } else {
#pragma unroll
            for (int t = 0; t < NV; ++t) v[t] = (R)0;
        }
#pragma unroll
        for (int t = 0; t < NV; ++t) cv[t][hc] = v[t];
    }
    __syncthreads();

    const Parts &P = D.pt;
    const int K = rp[NR];
    for (int k = tid; k < K; k += 256) {
        int lo = 0, hi = NR - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (rp[mid] <= k) lo = mid;
            else hi = mid - 1;
        }
        const int64_t i = rsrc[lo] + (k - rp[lo]);
        Stencil st;
        load_stencil<R>(P, i, st);
        // the stencil base is the particle's bin, inside this tile; the clamp
        // only keeps LDS indices in range for a particle already flagged as
        // having left the domain
        const int hx0 = min(max(st.b[0] - x0, 0), TX - 1), hy0 = min(max(st.b[1] - y0, 0), TY - 1),
                  hz0 = min(max(st.b[2] - z0, 0), TZ - 1);
        R acc[NV];
#pragma unroll
        for (int t = 0; t < NV; ++t) acc[t] = (R)0;
#pragma unroll 1
        for (int oz = 0; oz < 3; ++oz) {
#pragma unroll
            for (int oy = 0; oy < 3; ++oy) {
#pragma unroll
                for (int ox = 0; ox < 3; ++ox) {
                    const int hc = ((hz0 + oz) * HY + (hy0 + oy)) * HX + (hx0 + ox);
                    const R w = (R)(st.w[0][ox] * st.w[1][oy] * sel3(st.w[2], oz));
                    if (PASS == PASS_AM) {
#pragma unroll
                        for (int b = 0; b < 3; ++b) acc[b] += w * cv[b][hc];
                    } else if (PASS == PASS_AML) {
#pragma unroll
                        for (int b = 0; b < 3; ++b) {
                            acc[b] += w * cv[b][hc];
                            acc[3 + b] += w * cv[3 + b][hc];
                            acc[6 + b] += w * cv[6 + b][hc];
                        }
                    } else {
#pragma unroll
                        for (int b = 0; b < 3; ++b) {
                            acc[b] += w * cv[b][hc];
                            acc[3 + b] += w * cv[3 + b][hc];
                        }
                        acc[6] += w * cv[6][hc];
                    }
                }
            }
        }
        if (PASS == PASS_AM) {
            am_force<R>(D, i, acc);
        } else if (PASS == PASS_AML) {
            am_force<R>(D, i, acc);
            lift_force<R>(D, i, acc + 3, acc + 6);
        } else {
            drag_forces<R>(D, i, acc, acc + 3, acc[6], record);
        }
    }
}

// ---------------------------------------------------------------------------
// a8: DEM (Sec. 3.1.1) + lubrication (Sec. 3.1.3) forces of one substep.
// ---------------------------------------------------------------------------
// Pair and wall forces are evaluated in the compute type T (double in both
// storage forms: FP32 pair arithmetic was measured to cost ~5e-5 relative
// error per step in dense, lubrication-dominated packings). Positions,
// radii, the centre distance and the overlap (or gap) are FP64 whatever T
// is: the overlap is a small difference of O(1) lengths. In the
// FP32-deviation form the neighbour velocities, spins and masses come from
// the packed records, rounded to FP32.
template <typename T> struct PV {
    T r, m, d;
    double x[3];
    double rr;                  // radius, FP64
    T u[3], w[3];
};

template <typename T> __device__ __forceinline__ void cross3(const T a[3], const T b[3], T c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
template <typename T> __device__ __forceinline__ T dot3(const T a[3], const T b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// 1/x in FP64 from the hardware reciprocal estimate refined by two Newton
// steps (error below one ulp of the correctly rounded quotient for the
// positive, normal arguments used here): a third of the instructions of a
// full IEEE division
__device__ __forceinline__ double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float rcp64(float x) { return 1.0f / x; }

// Natural logarithm of a positive normal double: x = 2^k m with m in
// [1/sqrt 2, sqrt 2) and ln m = 2 atanh(s), s = (m - 1)/(m + 1), so that
// |s| <= 3 - 2 sqrt 2 = 0.1716, summed as the Taylor series of atanh through
// s^19 (the first omitted term is below 3e-17 of the sum). Within 2 ulp of
// the correctly rounded logarithm; about a third of the instructions of the
// general library logarithm, which also handles zero, negative, subnormal
// and non-finite arguments (the lubrication logarithm ln(<d>/2h) only sees
// gaps h >= h_min > 0).
__device__ __forceinline__ double log_pos(double x)
{
    double m = __builtin_amdgcn_frexp_mant(x);  // x = m 2^k, m in [1/2, 1)
    int k = __builtin_amdgcn_frexp_exp(x);
    if (m < M_SQRT1_2) {
        m += m;
        --k;
    }
    const double s = (m - 1.0) * rcp64(m + 1.0);
    const double z = s * s;
    double q = 1.0 / 19.0;
    q = fma(q, z, 1.0 / 17.0);
    q = fma(q, z, 1.0 / 15.0);
    q = fma(q, z, 1.0 / 13.0);
    q = fma(q, z, 1.0 / 11.0);
    q = fma(q, z, 1.0 / 9.0);
    q = fma(q, z, 1.0 / 7.0);
    q = fma(q, z, 1.0 / 5.0);
    q = fma(q, z, 1.0 / 3.0);
    const double t = s + s;
    return fma((double)k, M_LN2, fma(t * z, q, t));
}
__device__ __forceinline__ float log_pos(float x) { return logf(x); }

// spring-dashpot normal force and Coulomb-limited tangential force; torque
// about the centre is (d_i/2) n x F^t (the moment of F^t at the contact point)
template <typename T>
__device__ __forceinline__ void contact(const Phys &p, T delta, const T n[3], const T ur[3], T mij, T ri, T F[3],
                                        T Tq[3])
{
    const T kn = mij * (T)p.kn_per_m;
    const T xi = mij * (T)p.xi_per_m;
    const T urn_s = dot3(ur, n);
    T urn[3], urt[3], Fn[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        urn[a] = urn_s * n[a];
        urt[a] = ur[a] - urn[a];
        Fn[a] = -kn * delta * n[a] - xi * urn[a];
    }
    const T urt_n = sqrt(dot3(urt, urt));
    T Ft[3] = {(T)0, (T)0, (T)0};
    if (urt_n > (T)0) {
        const T fn_n = sqrt(dot3(Fn, Fn));
        const T mag = fmin((T)p.mu_c * fn_n, xi * urt_n) * rcp64(urt_n);
#pragma unroll
        for (int a = 0; a < 3; ++a) Ft[a] = -mag * urt[a];
    }
    T tq[3];
    cross3(n, Ft, tq);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        F[a] += Fn[a] + Ft[a];
        Tq[a] += ri * tq[a];
    }
}

// Eq. lubrication_force, applied for h < h_c with h := max(h, h_min) and,
// when lub_stab is set, h >= 3 pi mu <d>^2 dt_DEM / (8 r m_ij) with r = 1/4:
// the leading squeeze term then relaxes one pair by at most a quarter of
// its relative velocity per substep, so a sphere with a full shell of
// partners at the floor (up to (12 + 1)/2 times one pair's rate) stays
// below the explicit limit 2 - 2 C_am rho_f/rho_p; inv_dm = 1/<d>.
// With lub_contact = 0 only on the open gap (h > 0). The reduced mass is
// passed as m_ij = m_prod / m_sum.
template <typename T>
__device__ __forceinline__ void lubrication(const Phys &p, T h, T dm, T inv_dm, T m_prod, T m_sum, const T n[3],
                                            const T upr[3], T F[3])
{
    if (!(h < (T)p.h_c)) return;
    if (!p.lub_contact && !(h > (T)0)) return;  // open gap only
    const T mu = (T)p.mu;
    const T pi = (T)M_PI;
    T he = fmax(h, (T)p.h_min);
    if (p.lub_stab) {
        // he = max(he, c / (2 m_ij)) with m_ij = m_prod / m_sum, compared
        // without the division, which only the few pairs at the floor need
        const T c = (T)3 * pi * mu * dm * dm * (T)p.dt_dem * m_sum;
        if (he * ((T)2 * m_prod) < c) he = c * rcp64((T)2 * m_prod);
    }
    // 1/he and 1/(he + <d>) from one reciprocal
    const T q = rcp64(he * (he + dm));
    const T inv_he = (he + dm) * q;
    const T s = (T)2 * he * q;
    const T Lg = log_pos(dm * (T)0.5 * inv_he);
    const T asq = (T)1.5 * pi * mu * dm * (dm * (T)0.25 * inv_he + ((T)18 / (T)40) * Lg + ((T)9 / (T)84) * (he * inv_dm) * Lg);
    const T ash = (T)0.5 * pi * mu * dm * Lg * (dm + he) * (dm + he) / (T)4;
    const T un = dot3(upr, n);
#pragma unroll
    for (int a = 0; a < 3; ++a) F[a] += -asq * un * n[a] - ash * s * s * (upr[a] - un * n[a]);
}

// contact of the pair (i, j) at centre offset dx = x_j - x_i, |dx|^2 =
// dist2, when the spheres overlap
template <typename T>
__device__ __forceinline__ void pair_contact(const Phys &p, const PV<T> &pi, const PV<T> &pj, const double dx[3],
                                             double dist2, T F[3], T Tq[3])
{
    const double dist = sqrt(dist2);
    const T delta = (T)(pi.rr + pj.rr - dist);
    if (!(delta > (T)0)) return;
    const double inv = rcp64(dist);
    const T n[3] = {(T)(dx[0] * inv), (T)(dx[1] * inv), (T)(dx[2] * inv)};
    const T mij = pi.m * pj.m * rcp64(pi.m + pj.m);
    T s[3], ur[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) s[a] = pi.r * pi.w[a] + pj.r * pj.w[a];
    cross3(s, n, ur);
#pragma unroll
    for (int a = 0; a < 3; ++a) ur[a] += pi.u[a] - pj.u[a];
    contact(p, delta, n, ur, mij, pi.r, F, Tq);
}

// lubrication of the pair (i, j) at centre distance dist (unit normal n,
// overlap delta = r_i + r_j - dist)
template <typename T>
__device__ __forceinline__ void pair_lubrication(const Phys &p, const PV<T> &pi, const PV<T> &pj, const T n[3],
                                                 T delta, T F[3])
{
    // <d> = 2 d_i d_j / (d_i + d_j) and its inverse from one reciprocal
    const T sd = pi.d + pj.d, pd = pi.d * pj.d;
    const T q = rcp64(sd * pd);
    const T dm = (T)2 * pd * pd * q;
    const T inv_dm = (T)0.5 * sd * sd * q;
    const T upr[3] = {pi.u[0] - pj.u[0], pi.u[1] - pj.u[1], pi.u[2] - pj.u[2]};
    lubrication(p, -delta, dm, inv_dm, pi.m * pj.m, pi.m + pj.m, n, upr, F);
}

template <typename T>
__device__ __forceinline__ void wall_interaction(const Phys &p, const Geo &g, const PV<T> &pi, T F[3], T Tq[3])
{
    for (int a = 0; a < 3; ++a) {
        if (g.per[a]) continue;
        for (int side = 0; side < 2; ++side) {
            const double dist = side == 0 ? pi.x[a] : (double)g.n[a] - pi.x[a];
            T n[3] = {(T)0, (T)0, (T)0};
            n[a] = side == 0 ? (T)-1 : (T)1;
            const T delta = (T)(pi.rr - dist);
            if (delta > (T)0) {
                T s[3], ur[3];
#pragma unroll
                for (int b = 0; b < 3; ++b) s[b] = pi.r * pi.w[b];
                cross3(s, n, ur);
#pragma unroll
                for (int b = 0; b < 3; ++b) ur[b] += pi.u[b];
                contact(p, delta, n, ur, pi.m, pi.r, F, Tq);
            }
            if (p.use_lub) lubrication(p, -delta, (T)2 * pi.d, (T)0.5 * rcp64(pi.d), pi.m, (T)1, n, pi.u, F);
        }
    }
}

template <typename T> __device__ __forceinline__ void load_pv(const Parts &P, int64_t i, PV<T> &v)
{
    const int64_t cap = P.cap;
    const double d = P.d[i];
    v.d = (T)d;
    v.r = (T)(0.5 * d);
    v.rr = 0.5 * d;
    v.m = (T)(P.rho[i] * sphere_volume(d));
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        v.x[a] = P.x[a * cap + i];
        v.u[a] = (T)P.u[a * cap + i];
        v.w[a] = (T)P.w[a * cap + i];
    }
}

__device__ __forceinline__ void store_rec(DemRec *pk, int64_t i, const double x[3], const double u[3],
                                          const double w[3], double d, double rho)
{
    DemRec r;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.x[a] = x[a];
        r.u[a] = (float)u[a];
        r.w[a] = (float)w[a];
    }
    r.d = d;
    r.m = (float)(rho * sphere_volume(d));
    r.pad = 0.0f;
    const uint4 *src = reinterpret_cast<const uint4 *>(&r);
    uint4 *dst = reinterpret_cast<uint4 *>(pk + i);
#pragma unroll
    for (int k = 0; k < 4; ++k) dst[k] = src[k];
}

// a particle's DEM view from its 64-byte record: FP64 position and
// diameter, velocity, spin and mass as stored (FP32)
template <typename T> __device__ __forceinline__ void load_rec(const DemRec *pk, int64_t i, PV<T> &v)
{
    const uint4 *src = reinterpret_cast<const uint4 *>(pk + i);
    DemRec r;
    uint4 *dst = reinterpret_cast<uint4 *>(&r);
#pragma unroll
    for (int k = 0; k < 4; ++k) dst[k] = src[k];
    v.d = (T)r.d;
    v.r = (T)(0.5 * r.d);
    v.rr = 0.5 * r.d;
    v.m = (T)r.m;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        v.x[a] = r.x[a];
        v.u[a] = (T)r.u[a];
        v.w[a] = (T)r.w[a];
    }
}

// Once a step has flagged instability (non-finite or runaway particles),
// the domain's state is no longer meaningful and is reported at the next
// sync. The binning and neighbour-search kernels then do nothing: positions
// that are no longer finite all clamp into one cell, and sorting or
// scanning such a bin would take time quadratic in the particle count.
// (These kernels have no barriers, so a per-thread check is safe.)
__device__ __forceinline__ bool halted(const Desc &D) { return *(volatile const int *)D.flags != 0; }

__device__ __forceinline__ void min_image(const Geo &g, double dx[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (g.per[a]) {
            const double L = (double)g.n[a];
            dx[a] = dx[a] > 0.5 * L ? dx[a] - L : (dx[a] < -0.5 * L ? dx[a] + L : dx[a]);
        }
}

// Verlet lists (neighbour search for the sums of Eq. forces_collision,
// Eq. torques_collision and Eq. lubrication_force, which only reach
// (d_i + d_j)/2 + h_c). A list holds every particle within that reach plus a
// skin, as insertion indices sorted ascending, so the force sums run in an
// order that does not depend on when the list was built. Rebuilt only when a
// particle has moved more than (skin/2 - per-subcycle limit) since the build.
__global__ __launch_bounds__(kBlock) void k_nlist(Desc D)
{
    const Parts &P = D.pt;
    if (*P.need == 0 || halted(D)) return;
    const int64_t i = gidx();
    if (i >= P.np) return;
    const int64_t cap = P.cap;
    // lists are labelled by the slot at build time (particles keep their
    // label through the reorders and move little, so labels stay close to
    // slots and the label-indexed arrays are read almost in order)
    const int me = (int)i;
    const double xi0 = P.x[i], xi1 = P.x[cap + i], xi2 = P.x[2 * cap + i];
    const double ri = 0.5 * P.d[i];
    const double gap = (D.p.use_lub ? fmax(D.p.h_c, 0.0) : 0.0) + D.p.vskin;
    const int b0 = clampi((int)floor(xi0), 0, D.g.n[0] - 1);
    const int b1 = clampi((int)floor(xi1), 0, D.g.n[1] - 1);
    const int b2 = clampi((int)floor(xi2), 0, D.g.n[2] - 1);
    constexpr int kMaxR = 8;
    int cx[2 * kMaxR + 1], cy[2 * kMaxR + 1], cz[2 * kMaxR + 1];
    const int R = D.p.rbin;
    const int mx = axis_range(b0, R, D.g.n[0], D.g.per[0], cx, 2 * kMaxR + 1);
    const int my = axis_range(b1, R, D.g.n[1], D.g.per[1], cy, 2 * kMaxR + 1);
    const int mz = axis_range(b2, R, D.g.n[2], D.g.per[2], cz, 2 * kMaxR + 1);
    const bool run = mx >= 1 && cx[mx - 1] - cx[0] == mx - 1;
    const int nrun = run ? 1 : mx;
    int *L = P.nlist + (int64_t)me * P.nbr;
    int m = 0;
    for (int c2 = 0; c2 < mz; ++c2)
        for (int c1 = 0; c1 < my; ++c1)
            for (int c0 = 0; c0 < nrun; ++c0) {
                const int64_t bin = cidx(D.g, cx[c0], cy[c1], cz[c2]);
                const int p0 = D.b.start[bin];
                const int p1 = D.b.start[bin + (run ? mx : 1)];
                for (int j = p0; j < p1; ++j) {
                    if (j == i) continue;
                    double dx[3] = {P.x[j] - xi0, P.x[cap + j] - xi1, P.x[2 * cap + j] - xi2};
                    min_image(D.g, dx);
                    const double reach = ri + 0.5 * P.d[j] + gap;
                    if (dot3(dx, dx) >= reach * reach) continue;
                    if (m < P.nbr) {
                        // the neighbour's label (its slot now), kept in
                        // ascending insertion index, so the pair sums run in
                        // an order that does not depend on when the list was built
                        const int key = P.id[j];
                        int t = m - 1;
                        while (t >= 0 && P.id[L[t]] > key) {
                            L[t + 1] = L[t];
                            --t;
                        }
                        L[t + 1] = j;
                    }
                    ++m;
                }
            }
    if (m > P.nbr) {
        atomicOr(D.flags, FLAG_NLIST);
        m = P.nbr;
    }
    P.nnb[me] = m;
    P.xbuild[me] = xi0;
    P.xbuild[cap + me] = xi1;
    P.xbuild[2 * cap + me] = xi2;
    P.bslot[i] = me;
    P.slot_of[me] = (int)i;
}

// The neighbours' current slots, looked up once per subcycle, after the
// reordering that closed the last subcycle (and any rebuild), for the n_DEM
// force passes, which then read each neighbour's record without that
// dependent load (only with n_DEM >= kNslotMinSubsteps substeps, where that
// saves more than the lookup pass costs). kNslotLanes lanes share a row and
// take its entries four at a time (rows hold nbr entries, a multiple of
// four, so each quad is one aligned 16-byte load and store), up to the
// row's length only: the capacity is about three times the mean length,
// and a thread per quad of the whole capacity would mostly find nothing to
// do. The tail of a row's last quad is written as -1.
constexpr int kNslotMinSubsteps = 3;
__host__ __device__ __forceinline__ bool use_nslot(const Desc &D) { return D.p.n_dem >= kNslotMinSubsteps; }
constexpr int kNslotLanes = 8;

__global__ __launch_bounds__(kBlock) void k_nslot(Desc D)
{
    const Parts &P = D.pt;
    if (halted(D)) return;
    const uint64_t g = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t row = g / kNslotLanes;
    if (row >= (uint64_t)P.np) return;
    const int lane = (int)(g % kNslotLanes);
    const int n = P.nnb[row];
    const int64_t rb = (int64_t)row * P.nbr;
    for (int t = lane * 4; t < n; t += kNslotLanes * 4) {
        const int4 lab = *reinterpret_cast<const int4 *>(P.nlist + rb + t);
        int4 out;
        out.x = P.slot_of[lab.x];
        out.y = t + 1 < n ? P.slot_of[lab.y] : -1;
        out.z = t + 2 < n ? P.slot_of[lab.z] : -1;
        out.w = t + 3 < n ? P.slot_of[lab.w] : -1;
        *reinterpret_cast<int4 *>(P.nslot + rb + t) = out;
    }
}

// One semi-implicit Euler substep of particle i (R5: u and omega first,
// then x) under the contact and lubrication force F and torque Tq of the
// substep and the subcycle's frozen F_const, with the wall, skin and
// finiteness checks; rec: where the particle's new DEM record goes (none
// after the last substep of a subcycle, whose reorder rewrites every record).
__device__ __forceinline__ void integrate_particle(const Desc &D, int64_t i, int last, const double F[3],
                                                   const double Tq[3], DemRec *rec)
{
    const Parts &P = D.pt;
    const int64_t cap = P.cap;
    const double d = P.d[i];
    const double m = P.rho[i] * sphere_volume(d);
    const double I = m * d * d / 10.0;
    const double dt = D.p.dt_dem;
    double x[3];
    int bad = 0;
    double moved = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int64_t k = a * cap + i;
        const double u = P.u[k] + dt * (P.Fc[k] + F[a]) / m;
        P.u[k] = u;
        P.w[k] = P.w[k] + dt * Tq[a] / I;
        double xa = P.x[k] + dt * u;
        const double L = (double)D.g.n[a];
        if (D.g.per[a]) {
            if (xa >= L) xa -= L;
            else if (xa < 0.0) {
                xa += L;
                if (xa >= L) xa = 0.0;
            }
        } else if (!(xa > 0.0 && xa < L)) {
            bad |= FLAG_WALL;
        }
        if (!isfinite(xa) || !isfinite(u)) bad |= FLAG_NONFINITE;
        P.x[k] = xa;
        x[a] = xa;
        double dx = xa - P.xstart[k];
        if (D.g.per[a]) dx -= L * rint(dx / L);
        if (fabs(dx) > D.p.skin) bad |= FLAG_SKIN;
        if (last) P.a[k] = (u - P.ustart[k]) / D.p.dt_int;
        if (last) {
            double db = xa - P.xbuild[a * cap + P.bslot[i]];
            if (D.g.per[a]) db -= L * rint(db / L);
            moved = fmax(moved, fabs(db));
        }
    }
    if (bad) atomicOr(D.flags, bad);
    // the record feeds the next substep's pair loop
    if (rec && !last) {
        const double uu[3] = {P.u[i], P.u[cap + i], P.u[2 * cap + i]};
        const double ww[3] = {P.w[i], P.w[cap + i], P.w[2 * cap + i]};
        store_rec(rec, i, x, uu, ww, d, P.rho[i]);
    }
    // with at most `skin` per subcycle, rebuilding once any particle has moved
    // vskin/2 - skin keeps every pair within the list reach until the rebuild
    if (last && moved > 0.5 * D.p.vskin - D.p.skin) *P.need = 1;
    if (last) atomicAdd(&D.b.cnt[particle_cell(D.g, x[0], x[1], x[2])], 1);
}

// contact + lubrication force and torque on every particle from its list.
// The list is taken in runs of up to 64 entries. The first pass over a run
// evaluates the lubrication of every pair within reach and marks the
// overlapping ones; the second evaluates the contacts of the marked pairs
// only. Contacts are a small share of the pairs, and evaluated inline the
// whole wavefront would step through the contact code for almost every
// entry, since some lane nearly always has an overlap there. In the first
// pass entries are taken three at a time, their indices, slots and particle
// data requested together so that the memory latencies overlap. With
// NSLOT the neighbours' current slots come from the subcycle's refreshed
// copy of the list (k_nslot), saving a dependent load per neighbour;
// otherwise they are looked up from the labels here. Both sums
// run in list order; lubrication, contacts and the walls are summed apart
// and added at the end.

template <typename T, bool REC, bool NSLOT, bool FUSE>
__global__ __launch_bounds__(kBlock) void k_dem_force(Desc D, int last, int odd)
{
    static_assert(!FUSE || REC, "the fused substep reads packed records only");
    const Parts &P = D.pt;
    const int64_t v = gidx();
    if (v == 0) *P.need = 0;  // lists are current for this subcycle
    if (v >= P.np) return;
    const int64_t i = D.t.dem_order ? (int64_t)D.o.porder[v] : v;
    // FUSE: substeps alternate between the two record buffers, reading the
    // records of the substep's start and writing the integrated ones to the
    // other buffer, so that no thread sees another's update
    const DemRec *src = FUSE && odd ? P.pk2 : P.pk;
    PV<T> pi;
    if constexpr (REC) load_rec(src, i, pi);
    else load_pv(P, i, pi);
    T F[3] = {(T)0, (T)0, (T)0}, Tq[3] = {(T)0, (T)0, (T)0}, Fl[3] = {(T)0, (T)0, (T)0};
    const double gap = D.p.use_lub ? fmax(D.p.h_c, 0.0) : 0.0;
    const int me = P.bslot[i];
    const int n = P.nnb[me];
    // the neighbours' slots (NSLOT) or labels, in list order
    const int *S = (NSLOT ? P.nslot : P.nlist) + (int64_t)me * P.nbr;
    constexpr int kChunk = 3;
    for (int s0 = 0; s0 < n; s0 += 64) {
        const int s1 = min(n, s0 + 64);
        uint64_t touch = 0;
        for (int t0 = s0; t0 < s1; t0 += kChunk) {
            int js[kChunk];
#pragma unroll
            for (int c = 0; c < kChunk; ++c)
                js[c] = t0 + c < s1 ? (NSLOT ? S[t0 + c] : P.slot_of[S[t0 + c]]) : (int)i;
            PV<T> pj[kChunk];
#pragma unroll
            for (int c = 0; c < kChunk; ++c) {
                if constexpr (REC) load_rec(src, js[c], pj[c]);
                else load_pv(P, js[c], pj[c]);
            }
#pragma unroll
            for (int c = 0; c < kChunk; ++c) {
                if (t0 + c >= s1) break;
                double dx[3] = {pj[c].x[0] - pi.x[0], pj[c].x[1] - pi.x[1], pj[c].x[2] - pi.x[2]};
                min_image(D.g, dx);
                const double reach = pi.rr + pj[c].rr + gap;
                const double dist2 = dot3(dx, dx);
                if (dist2 >= reach * reach) continue;
                const double dist = sqrt(dist2);
                const T delta = (T)(pi.rr + pj[c].rr - dist);
                if (delta > (T)0) touch |= 1ull << (t0 + c - s0);
                if (D.p.use_lub) {
                    const double inv = rcp64(dist);
                    const T nv[3] = {(T)(dx[0] * inv), (T)(dx[1] * inv), (T)(dx[2] * inv)};
                    pair_lubrication(D.p, pi, pj[c], nv, delta, Fl);
                }
            }
        }
        while (touch) {
            const int t = __builtin_ctzll(touch);
            touch &= touch - 1;
            PV<T> pj;
            const int64_t j = NSLOT ? S[s0 + t] : P.slot_of[S[s0 + t]];
            if constexpr (REC) load_rec(src, j, pj);
            else load_pv(P, j, pj);
            double dx[3] = {pj.x[0] - pi.x[0], pj.x[1] - pi.x[1], pj.x[2] - pi.x[2]};
            min_image(D.g, dx);
            pair_contact(D.p, pi, pj, dx, dot3(dx, dx), F, Tq);
        }
    }
    wall_interaction(D.p, D.g, pi, F, Tq);
    const int64_t cap = P.cap;
    const double Fs[3] = {(double)(F[0] + Fl[0]), (double)(F[1] + Fl[1]), (double)(F[2] + Fl[2])};
    const double Ts[3] = {(double)Tq[0], (double)Tq[1], (double)Tq[2]};
    if constexpr (FUSE) {
        integrate_particle(D, i, last, Fs, Ts, odd ? P.pk : P.pk2);
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            P.Fdem[a * cap + i] = Fs[a];
            P.Tdem[a * cap + i] = Ts[a];
        }
    }
}

// Blocked processing order of the DEM force pass (see Order): block row r
// = (block, lz, ly) with blocks row-major over the domain and rows y-fastest
// inside a block; its cells are x0 <= x < x1 of row (y, z). Rows of the
// padded last blocks that fall outside the domain are empty.
__device__ __forceinline__ bool order_row(const Desc &D, int64_t r, int &x0, int &x1, int &y, int &z)
{
    const Order &O = D.o;
    const int64_t per = (int64_t)O.ob[1] * O.ob[2];
    const int64_t blk = r / per, lr = r - blk * per;
    const int ly = (int)(lr % O.ob[1]), lz = (int)(lr / O.ob[1]);
    const int bxi = (int)(blk % O.nb[0]);
    const int byi = (int)((blk / O.nb[0]) % O.nb[1]);
    const int bzi = (int)(blk / ((int64_t)O.nb[0] * O.nb[1]));
    y = byi * O.ob[1] + ly;
    z = bzi * O.ob[2] + lz;
    x0 = bxi * O.ob[0];
    x1 = min(x0 + O.ob[0], D.g.n[0]);
    return y < D.g.n[1] && z < D.g.n[2];
}

__device__ __forceinline__ int order_row_count(const Desc &D, int x0, int x1, int y, int z, int &s0)
{
    s0 = D.b.start[cidx(D.g, x0, y, z)];
    return D.b.start[cidx(D.g, x1 - 1, y, z) + 1] - s0;
}

// particles per block row, scanned within blocks of kScanPerBlock rows
__global__ __launch_bounds__(kBlock) void k_order_scan(Desc D)
{
    __shared__ int wsum[kBlock / 64];
    const int64_t n = D.o.nrows;
    const int64_t base = (int64_t)blockIdx.x * kScanPerBlock + (int64_t)threadIdx.x * kScanItems;
    int v[kScanItems];
    int tot = 0;
#pragma unroll
    for (int t = 0; t < kScanItems; ++t) {
        int x0, x1, y, z, s0;
        v[t] = (base + t < n && order_row(D, base + t, x0, x1, y, z)) ? order_row_count(D, x0, x1, y, z, s0) : 0;
        tot += v[t];
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int incl = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int run = incl - tot, btot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        const int ws = wsum[w];
        if (w < wv) run += ws;
        btot += ws;
    }
#pragma unroll
    for (int t = 0; t < kScanItems; ++t) {
        if (base + t < n) D.o.rowoff[base + t] = run;
        run += v[t];
    }
    if (threadIdx.x == kBlock - 1) D.o.rowsum[blockIdx.x] = btot;
}

// porder[offset of row r + k] = first slot of row r + k
__global__ __launch_bounds__(kBlock) void k_order_fill(Desc D)
{
    const int64_t r = gidx();
    if (r >= D.o.nrows || halted(D)) return;
    int x0, x1, y, z, s0;
    if (!order_row(D, r, x0, x1, y, z)) return;
    const int cnt = order_row_count(D, x0, x1, y, z, s0);
    const int off = D.o.rowoff[r] + D.o.rowsum[r / kScanPerBlock];
    for (int k = 0; k < cnt; ++k) D.o.porder[off + k] = s0 + k;
}

// semi-implicit Euler with the fluid forces frozen (Sec. 3.3); periodic wrap;
// at the last substep of a subcycle: du_p/dt over the subcycle and bin count
__global__ __launch_bounds__(kBlock) void k_integrate(Desc D, int last)
{
    const int64_t i = gidx();
    const Parts &P = D.pt;
    if (i >= P.np) return;
    const int64_t cap = P.cap;
    const double F[3] = {P.Fdem[i], P.Fdem[cap + i], P.Fdem[2 * cap + i]};
    const double Tq[3] = {P.Tdem[i], P.Tdem[cap + i], P.Tdem[2 * cap + i]};
    integrate_particle(D, i, last, F, Tq, P.pk);
}

__global__ __launch_bounds__(kBlock) void k_bin_count(Desc D)
{
    const int64_t i = gidx();
    const Parts &P = D.pt;
    if (i >= P.np || halted(D)) return;
    const int64_t cap = P.cap;
    atomicAdd(&D.b.cnt[particle_cell(D.g, P.x[i], P.x[cap + i], P.x[2 * cap + i])], 1);
}

// exclusive scan of cnt into start (block level); resets cnt
__global__ __launch_bounds__(kBlock) void k_scan_block(Desc D)
{
    __shared__ int wsum[kBlock / 64];
    const int64_t nc = D.g.nc;
    const int64_t base = (int64_t)blockIdx.x * kScanPerBlock + (int64_t)threadIdx.x * kScanItems;
    static_assert(kScanItems == 8, "two 16-byte vectors per thread");
    // a thread's 8 counts are 32-byte aligned: two vector loads, scalar
    // loads only for the last, ragged chunk
    const bool full = base + kScanItems <= nc;
    int v[kScanItems];
    if (full) {
        const int4 a = *reinterpret_cast<const int4 *>(D.b.cnt + base);
        const int4 b = *reinterpret_cast<const int4 *>(D.b.cnt + base + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
    } else {
#pragma unroll
        for (int t = 0; t < kScanItems; ++t) v[t] = base + t < nc ? D.b.cnt[base + t] : 0;
    }
    int tot = 0;
#pragma unroll
    for (int t = 0; t < kScanItems; ++t) tot += v[t];
    // wavefront-shuffle scan, then the wavefront totals (one barrier)
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int incl = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int run = incl - tot, btot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        const int ws = wsum[w];
        if (w < wv) run += ws;
        btot += ws;
    }
    int o[kScanItems];
#pragma unroll
    for (int t = 0; t < kScanItems; ++t) {
        o[t] = run;
        run += v[t];
    }
    if (full) {
        *reinterpret_cast<int4 *>(D.b.loc + base) = make_int4(o[0], o[1], o[2], o[3]);
        *reinterpret_cast<int4 *>(D.b.loc + base + 4) = make_int4(o[4], o[5], o[6], o[7]);
        *reinterpret_cast<int4 *>(D.b.cnt + base) = make_int4(0, 0, 0, 0);
        *reinterpret_cast<int4 *>(D.b.cnt + base + 4) = make_int4(0, 0, 0, 0);
    } else {
#pragma unroll
        for (int t = 0; t < kScanItems; ++t)
            if (base + t < nc) {
                D.b.loc[base + t] = o[t];
                D.b.cnt[base + t] = 0;
            }
    }
    if (threadIdx.x == kBlock - 1) D.b.bsum[blockIdx.x] = btot;
}

// exclusive scan of the block sums, one block of 1024 threads
__global__ __launch_bounds__(1024) void k_scan_top(int *bsum, int nb, int *total)
{
    __shared__ int sh[1024];
    const int per = (nb + 1023) / 1024;
    const int b0 = threadIdx.x * per;
    int tot = 0;
    for (int t = 0; t < per; ++t)
        if (b0 + t < nb) tot += bsum[b0 + t];
    sh[threadIdx.x] = tot;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int add = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    int run = sh[threadIdx.x] - tot;
    for (int t = 0; t < per; ++t)
        if (b0 + t < nb) {
            const int v = bsum[b0 + t];
            bsum[b0 + t] = run;
            run += v;
        }
    if (threadIdx.x == 1023) *total = sh[1023];
}

// slot range start of bin c from the block-local prefix and the block offset
__device__ __forceinline__ int bin_start(const Bins &B, int64_t c)
{
    return B.loc[c] + B.bsum[c / kScanPerBlock];
}

__global__ __launch_bounds__(kBlock) void k_place(Desc D)
{
    const int64_t i = gidx();
    const Parts &P = D.pt;
    if (i >= P.np || halted(D)) return;
    const int64_t cap = P.cap;
    const int64_t c = particle_cell(D.g, P.x[i], P.x[cap + i], P.x[2 * cap + i]);
    const int pos = bin_start(D.b, c) + atomicAdd(&D.b.cnt[c], 1);
    D.b.list[pos] = (int)i;
}

// order each bin by insertion index (so that every sum over a bin runs in a
// history-independent order), write the final bin offsets, reset the counts
__global__ __launch_bounds__(kBlock) void k_cellsort(Desc D)
{
    const int64_t nc = D.g.nc;
    const int64_t c = gidx();
    if (c >= nc || halted(D)) return;
    D.b.cnt[c] = 0;
    const int p0 = bin_start(D.b, c), p1 = c + 1 < nc ? bin_start(D.b, c + 1) : D.b.start[nc];
    D.b.start[c] = p0;
    const int *id = D.pt.id;
    int *L = D.b.list;
    for (int a = p0 + 1; a < p1; ++a) {
        const int v = L[a];
        const int key = id[v];
        int b = a - 1;
        while (b >= p0 && id[L[b]] > key) {
            L[b + 1] = L[b];
            --b;
        }
        L[b + 1] = v;
    }
}

// gather the particle state into bin order (slot s <- list[s]) and evaluate
// the kernel stencils of the new positions
// moves the particle bound for slot s into the permutation targets and
// evaluates its kernel stencil; returns what the fused added-mass pass needs
__device__ __forceinline__ void permute_slot(const Desc &D, int64_t s, double x[3], double u[3], double acc[3],
                                             double &d, Stencil &st)
{
    const Parts &P = D.pt;
    const int64_t cap = P.cap;
    const int src = D.b.list[s];
    double w[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        x[a] = P.x[a * cap + src];
        u[a] = P.u[a * cap + src];
        w[a] = P.w[a * cap + src];
        acc[a] = P.a[a * cap + src];
        P.x2[a * cap + s] = x[a];
        P.u2[a * cap + s] = u[a];
        P.w2[a * cap + s] = w[a];
        P.a2[a * cap + s] = acc[a];
        int b;
        double wt[3];
        axis_weights(x[a], D.g.n[a], D.g.per[a], b, wt);
        P.sb[a * cap + s] = b;
        st.b[a] = b;
        if (P.swf) {
#pragma unroll
            for (int o = 0; o < 3; ++o) {
                P.swf[(3 * a + o) * cap + s] = (float)wt[o];
                st.w[a][o] = (double)(float)wt[o];
            }
        } else {
#pragma unroll
            for (int o = 0; o < 3; ++o) {
                P.sw[(3 * a + o) * cap + s] = wt[o];
                st.w[a][o] = wt[o];
            }
        }
    }
    d = P.d[src];
    const double rho = P.rho[src];
    P.d2[s] = d;
    P.rho2[s] = rho;
    P.id2[s] = P.id[src];
    const int lab = P.bslot[src];
    P.bslot2[s] = lab;
    P.slot_of[lab] = (int)s;
    if (P.pk2) store_rec(P.pk2, s, x, u, w, d, rho);
}

__global__ __launch_bounds__(kBlock) void k_permute(Desc D)
{
    const int64_t s = gidx();
    if (s >= D.pt.np || halted(D)) return;
    double x[3], u[3], a[3], d;
    Stencil st;
    permute_slot(D, s, x, u, a, d, st);
}

// the permutation followed by the next subcycle's added-mass force of the
// particle (a4 without lift): the stencil, position, velocity and du_p/dt are
// already in registers. The stored-precision weights and the summation order
// are those of k_part_am, so the forces are bit-identical.
template <typename R>
__global__ __launch_bounds__(kBlock) void k_permute_am(Desc D, Cells<R> C)
{
    const int64_t s = gidx();
    if (s >= D.pt.np || halted(D)) return;
    double x[3], u[3], a[3], d;
    Stencil st;
    permute_slot(D, s, x, u, a, d, st);
    R Du[3] = {(R)0, (R)0, (R)0};
    interp_dudt<R>(D, C, st, Du);
    am_store<R>(D, s, Du, d, a, u, x);
}

// ---------------------------------------------------------------------------
// a10: fused GNS-LBM collide + stream (Eq. LBM_Equation, Eq. LBM_EQ,
// Eq. Forcing, Eq. MacVel), push form: reads the post-stream PDFs of its own
// cell, writes the post-collision values to x + c_q. Links leaving through a
// wall reflect in place into the opposite direction (half-way bounce-back).
// ---------------------------------------------------------------------------
// GNS-BGK collision with Guo forcing of one cell (the post-collision values
// of all 19 directions, before streaming)
// Per-cell relaxation time tau_e = tau_* + tau_t (Eq. tau_e; Alg. 1, before
// the GNS-LBM step), in the storage precision R:
//  - Eilers (Eq. visc_eilers with the denominator 1 - eps_p/eps_cp of Eilers'
//    form; [mu] = 2.5, eps_cp = 0.64) through Eq. visc_tau_*:
//    tau_* = 1/2 + (tau - 1/2) (1 + 1.25 eps_p/(1 - eps_p/0.64))^2;
//  - Smagorinsky (Eq. visc_turb, C_s = 0.1, dx = 1): tau_t is the positive
//    root of tau_t^2 + tau_* tau_t = C_s^2 Qbar/(2 rho c_s^4), Qbar =
//    sqrt(2 sum Q_ab Q_ab), Q_ab = sum_q c_qa c_qb (f_q - f_q^eq).
template <typename R>
__device__ __forceinline__ R relax_time(const Desc &D, R ep, R rho, const R f[19], const R feq[19])
{
    const R one = (R)1;
    R tau = (R)D.p.tau;
    if (D.p.use_eilers) {
        const R b = one + (R)1.25 * ep / (one - ep / (R)0.64);
        tau = (R)0.5 + ((R)D.p.tau - (R)0.5) * b * b;
    }
    if (D.p.use_les) {
        R qxx = 0, qyy = 0, qzz = 0, qxy = 0, qxz = 0, qyz = 0;
#pragma unroll
        for (int q = 1; q < 19; ++q) {
            const R n = f[q] - feq[q];
            if (CX(q) != 0) qxx += n;
            if (CY(q) != 0) qyy += n;
            if (CZ(q) != 0) qzz += n;
            if (CX(q) * CY(q) > 0) qxy += n; else if (CX(q) * CY(q) < 0) qxy -= n;
            if (CX(q) * CZ(q) > 0) qxz += n; else if (CX(q) * CZ(q) < 0) qxz -= n;
            if (CY(q) * CZ(q) > 0) qyz += n; else if (CY(q) * CZ(q) < 0) qyz -= n;
        }
        const R qq = qxx * qxx + qyy * qyy + qzz * qzz + (R)2 * (qxy * qxy + qxz * qxz + qyz * qyz);
        const R qbar = sqrt((R)2 * qq);
        // C_s^2 Qbar / (2 rho c_s^4) with C_s^2 = 0.01, 1/c_s^4 = 9
        const R rhs = (R)0.045 * qbar / rho;
        tau += (R)0.5 * (sqrt(tau * tau + (R)4 * rhs) - tau);
    }
    return tau;
}

template <typename R, bool VISC>
__device__ __forceinline__ void collide_cell(const Desc &D, const Cells<R> &C, int64_t c, R post[19], int &bad)
{
    const int64_t nc = D.g.nc;
    R f[19];
#pragma unroll
    for (int q = 0; q < 19; ++q) f[q] = C.df_src[q * nc + c];
    R r = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        r += f[q];
        if (CX(q) > 0) jx += f[q]; else if (CX(q) < 0) jx -= f[q];
        if (CY(q) > 0) jy += f[q]; else if (CY(q) < 0) jy -= f[q];
        if (CZ(q) > 0) jz += f[q]; else if (CZ(q) < 0) jz -= f[q];
    }
    const R one = (R)1;
    const R rho = one + r;
    const R fx = C.facc[c], fy = C.facc[nc + c], fz = C.facc[2 * nc + c];
    const R half = (R)0.5;
    const R ux = (jx + half * fx) / rho, uy = (jy + half * fy) / rho, uz = (jz + half * fz) / rho;
    const R eps = one - C.epsp[c];
    const R ieps = one / eps;
    const R uu = ux * ux + uy * uy + uz * uz;
    // non-finite PDFs make rho or u non-finite; |u| > 0.1 leaves the low-Mach
    // range in which the equilibrium expansion holds
    if (!isfinite(rho) || !isfinite(uu)) bad = FLAG_FLUID_NONFINITE;
    else if (uu > (R)0.01) bad = FLAG_MACH;
    if (VISC) {
        R feq[19];
#pragma unroll
        for (int q = 0; q < 19; ++q) {
            const R cu = (R)CX(q) * ux + (R)CY(q) * uy + (R)CZ(q) * uz;
            const R w = (R)WQ(q);
            feq[q] = w * r + w * rho * ((R)3 * cu + (R)4.5 * cu * cu * ieps - (R)1.5 * uu * ieps);
        }
        const R tau = relax_time<R>(D, C.epsp[c], rho, f, feq);
        const R om = one / tau;
        const R pre = one - half / tau;
#pragma unroll
        for (int q = 0; q < 19; ++q) {
            const R cu = (R)CX(q) * ux + (R)CY(q) * uy + (R)CZ(q) * uz;
            const R w = (R)WQ(q);
            const R gx = (R)3 * (R)CX(q) - (R)3 * ux * ieps + (R)9 * cu * (R)CX(q) * ieps;
            const R gy = (R)3 * (R)CY(q) - (R)3 * uy * ieps + (R)9 * cu * (R)CY(q) * ieps;
            const R gz = (R)3 * (R)CZ(q) - (R)3 * uz * ieps + (R)9 * cu * (R)CZ(q) * ieps;
            const R F = w * pre * (gx * fx + gy * fy + gz * fz);
            post[q] = f[q] + (feq[q] - f[q]) * om + F;
        }
        return;
    }
    const R om = (R)D.p.omega;
    const R pre = (R)(1.0 - 0.5 / D.p.tau);
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        const R cu = (R)CX(q) * ux + (R)CY(q) * uy + (R)CZ(q) * uz;
        const R w = (R)WQ(q);
        const R feq = w * r + w * rho * ((R)3 * cu + (R)4.5 * cu * cu * ieps - (R)1.5 * uu * ieps);
        const R gx = (R)3 * (R)CX(q) - (R)3 * ux * ieps + (R)9 * cu * (R)CX(q) * ieps;
        const R gy = (R)3 * (R)CY(q) - (R)3 * uy * ieps + (R)9 * cu * (R)CY(q) * ieps;
        const R gz = (R)3 * (R)CZ(q) - (R)3 * uz * ieps + (R)9 * cu * (R)CZ(q) * ieps;
        const R F = w * pre * (gx * fx + gy * fy + gz * fz);
        post[q] = f[q] + (feq - f[q]) * om + F;
    }
}

// push streaming: direction q of cell (i, j, k) goes to (i, j, k) + c_q,
// wrapped on periodic axes; where it would leave through a wall it returns
// into the opposite direction of the same cell (half-way bounce-back)
template <typename R, bool VISC>
__global__ __launch_bounds__(kBlock) void k_stream_collide(Desc D, Cells<R> C)
{
    const int64_t nc = D.g.nc;
    const int64_t c = gidx();
    if (c == 0) *D.stepc += 1;
    if (c >= nc) return;
    int i, j, k;
    cell_coords(D.g, c, i, j, k);
    R post[19];
    int bad = 0;
    collide_cell<R, VISC>(D, C, c, post, bad);
    if (bad) atomicOr(D.flags, bad);
    const bool wall_x = !D.g.per[0], wall_y = !D.g.per[1], wall_z = !D.g.per[2];
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        int t0 = i + CX(q), t1 = j + CY(q), t2 = k + CZ(q);
        bool wall = false;
        if (CX(q) != 0 && (t0 < 0 || t0 >= D.g.n[0])) {
            if (wall_x) wall = true; else t0 = t0 < 0 ? t0 + D.g.n[0] : t0 - D.g.n[0];
        }
        if (CY(q) != 0 && (t1 < 0 || t1 >= D.g.n[1])) {
            if (wall_y) wall = true; else t1 = t1 < 0 ? t1 + D.g.n[1] : t1 - D.g.n[1];
        }
        if (CZ(q) != 0 && (t2 < 0 || t2 >= D.g.n[2])) {
            if (wall_z) wall = true; else t2 = t2 < 0 ? t2 + D.g.n[2] : t2 - D.g.n[2];
        }
        if (wall) C.df_dst[OPP(q) * nc + c] = post[q];
        else C.df_dst[q * nc + cidx(D.g, t0, t1, t2)] = post[q];
    }
}

// ---------------------------------------------------------------------------
// reductions for the diagnostics (two passes, fixed order: deterministic)
// per-block partials: [0] sum drho, [1..3] sum j, [4] sum eps, [5] min eps,
// [6] sum u_f,z, [7] max |u_bar|, [8..10] sum m u, [11] sum u_z
// ---------------------------------------------------------------------------
constexpr int kDiag = kDiagValues;

template <typename R>
__global__ __launch_bounds__(kBlock) void k_diag(Desc D, Cells<R> C, const R *df, double *part)
{
    __shared__ double sh[kDiag][kBlock];
    const int64_t nc = D.g.nc, np = D.pt.np, cap = D.pt.cap;
    double acc[kDiag] = {0, 0, 0, 0, 0, 1e300, 0, 0, 0, 0, 0, 0};
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t c = gidx(); c < nc; c += stride) {
        double r = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
        for (int q = 0; q < 19; ++q) {
            const double f = (double)df[q * nc + c];
            r += f;
            jx += CX(q) * f;
            jy += CY(q) * f;
            jz += CZ(q) * f;
        }
        const double e = 1.0 - (double)C.epsp[c];
        const double rho = 1.0 + r;
        const double ub0 = (jx + 0.5 * e * D.p.fb[0]) / rho;
        const double ub1 = (jy + 0.5 * e * D.p.fb[1]) / rho;
        const double ub2 = (jz + 0.5 * e * D.p.fb[2]) / rho;
        acc[0] += r;
        acc[1] += jx;
        acc[2] += jy;
        acc[3] += jz;
        acc[4] += e;
        acc[5] = fmin(acc[5], e);
        acc[6] += ub2 / e;
        acc[7] = fmax(acc[7], sqrt(ub0 * ub0 + ub1 * ub1 + ub2 * ub2));
    }
    for (int64_t i = gidx(); i < np; i += stride) {
        const double m = D.pt.rho[i] * sphere_volume(D.pt.d[i]);
        acc[8] += m * D.pt.u[i];
        acc[9] += m * D.pt.u[cap + i];
        acc[10] += m * D.pt.u[2 * cap + i];
        acc[11] += D.pt.u[2 * cap + i];
    }
#pragma unroll
    for (int t = 0; t < kDiag; ++t) sh[t][threadIdx.x] = acc[t];
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (threadIdx.x < (unsigned)off) {
#pragma unroll
            for (int t = 0; t < kDiag; ++t) {
                const double a = sh[t][threadIdx.x], b = sh[t][threadIdx.x + off];
                sh[t][threadIdx.x] = t == 5 ? fmin(a, b) : (t == 7 ? fmax(a, b) : a + b);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < kDiag) part[(int64_t)blockIdx.x * kDiag + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_diag_final(const double *part, int nblk, double *out)
{
    const int t = threadIdx.x;
    if (t >= kDiag) return;
    double a = t == 5 ? 1e300 : 0.0;
    for (int b = 0; b < nblk; ++b) {
        const double v = part[(int64_t)b * kDiag + t];
        a = t == 5 ? fmin(a, v) : (t == 7 ? fmax(a, v) : a + v);
    }
    out[t] = a;
}

template <typename R>
__global__ void k_zero(R *p, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = (R)0;
}

template <typename A, typename B>
__global__ void k_convert(const A *src, B *dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = (B)src[i];
}

// stored solid fraction -> fluid volume fraction 1 - eps_p, FP64
template <typename A> __global__ void k_fluid_fraction(const A *src, double *dst, int64_t nc)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += stride)
        dst[c] = 1.0 - (double)src[c];
}

// [nc][4] -> [3][nc] doubles
template <typename A> __global__ void k_vec4_to_soa(const A *src, double *dst, int64_t nc)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += stride)
#pragma unroll
        for (int b = 0; b < 3; ++b) dst[b * nc + c] = (double)src[4 * c + b];
}

__global__ void k_set_step(long long *s, long long v) { *s = v; }
__global__ void k_set_int(int *p, int v) { *p = v; }

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblocks(int64_t n, int64_t per = kBlock)
{
    return (unsigned)((n + per - 1) / per);
}
static inline unsigned grid_stride_blocks(int64_t n)
{
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// Residency of the streaming cell passes: unused dynamic LDS caps the
// workgroups per CU (160 KB of LDS per CU); -1 is the measured default (4
// workgroups of 256 threads, 4 waves per SIMD, for the FP32 stream-collide)
static inline unsigned cell_lds_bytes(int cell_waves, unsigned dflt)
{
    if (cell_waves < 0) return dflt;
    if (cell_waves == 0) return 0u;
    return (160u * 1024u / (unsigned)cell_waves) & ~255u;
}
template <typename R> void launch_moments(const Desc &D, const Cells<R> &C, hipStream_t s)
{
    hipLaunchKernelGGL(k_moments<R>, dim3(nblocks(D.g.nc)), dim3(kBlock), cell_lds_bytes(D.t.cell_waves, 0u), s, D,
                       C);
}
template <typename R> void launch_cellfields(const Desc &D, const Cells<R> &C, hipStream_t s)
{
    hipLaunchKernelGGL(k_cellfields<R>, dim3(nblocks(D.g.nc)), dim3(kBlock), 0, s, D, C);
}
template <typename R> void launch_curl(const Desc &D, const Cells<R> &C, hipStream_t s)
{
    hipLaunchKernelGGL(k_curl<R>, dim3(nblocks(D.g.nc)), dim3(kBlock), 0, s, D, C);
}
// added-mass pass: one thread per particle (its 3-component stencil reads
// are cheap enough that LDS staging of the halo does not pay). With lift it
// reads 9 components per stencil cell and uses LDS tiles (16x4x8 cells in
// FP32, 16x4x4 in FP64 to stay within 64 KiB of LDS), or one thread per
// particle under gather variant 3.
template <typename R> void launch_part_am(const Desc &D, const Cells<R> &C, hipStream_t s)
{
    if (D.pt.np == 0) return;
    if (!D.p.use_lift) {
        hipLaunchKernelGGL((k_part_am<R, false>), dim3(nblocks(D.pt.np)), dim3(kBlock), 0, s, D, C);
        return;
    }
    if (D.t.gather == 3) {
        hipLaunchKernelGGL((k_part_am<R, true>), dim3(nblocks(D.pt.np)), dim3(kBlock), 0, s, D, C);
        return;
    }
    constexpr int TZ = sizeof(R) == 4 ? 8 : 4;
    dim3 grid((D.g.n[0] + 15) / 16, (D.g.n[1] + 3) / 4, (D.g.n[2] + TZ - 1) / TZ);
    hipLaunchKernelGGL((k_part_tile<R, PASS_AML, 16, 4, TZ>), grid, dim3(256), 0, s, D, C, 0);
}
// gather variants (chosen per domain by the autotuner, else by particle
// density): 0 tiles of 16x4x8 cells (two per thread, up to 256 staged
// particles); 1 16x4x4 (384); 2 8x4x4 (640); 3 one thread per cell from
// global memory; 4 16x4x16 (four per thread, 512). All give bit-identical
// results: every cell sums its bins in the same order and precision.
// Periodic axes thinner than 3 cells use the per-cell gather.
template <typename R, int MODE> void launch_gather(const Desc &D, const Cells<R> &C, hipStream_t s)
{
    const bool thin = (D.g.per[0] && D.g.n[0] < 3) || (D.g.per[1] && D.g.n[1] < 3) || (D.g.per[2] && D.g.n[2] < 3);
    if (thin || D.t.gather == 3) {
        hipLaunchKernelGGL((k_gather_cells<R, MODE>), dim3(nblocks(D.g.nc)), dim3(kBlock), 0, s, D, C);
        return;
    }
    int v = D.t.gather;
    if (v < 0 || v >= kGatherVariants) {
        const double density = D.g.nc > 0 ? (double)D.pt.np / (double)D.g.nc : 0.0;
        v = density < 0.3 ? 0 : (density < 1.0 ? 1 : 2);
    }
    if (v == 0) {
        dim3 grid((D.g.n[0] + 15) / 16, (D.g.n[1] + 3) / 4, (D.g.n[2] + 7) / 8);
        hipLaunchKernelGGL((k_gather_tile<R, MODE, 16, 4, 4, 2, 256>), grid, dim3(256), 0, s, D, C);
    } else if (v == 1) {
        dim3 grid((D.g.n[0] + 15) / 16, (D.g.n[1] + 3) / 4, (D.g.n[2] + 3) / 4);
        hipLaunchKernelGGL((k_gather_tile<R, MODE, 16, 4, 4, 1, 384>), grid, dim3(256), 0, s, D, C);
    } else if (v == 2) {
        dim3 grid((D.g.n[0] + 7) / 8, (D.g.n[1] + 3) / 4, (D.g.n[2] + 3) / 4);
        hipLaunchKernelGGL((k_gather_tile<R, MODE, 8, 4, 4, 1, 640>), grid, dim3(128), 0, s, D, C);
    } else {
        dim3 grid((D.g.n[0] + 15) / 16, (D.g.n[1] + 3) / 4, (D.g.n[2] + 15) / 16);
        hipLaunchKernelGGL((k_gather_tile<R, MODE, 16, 4, 4, 4, 512>), grid, dim3(256), 0, s, D, C);
    }
}
template <typename R> void launch_gather_am(const Desc &D, const Cells<R> &C, hipStream_t s)
{
    launch_gather<R, MODE_AM>(D, C, s);
}
// drag/pressure pass: LDS tiles, or one thread per particle reading its
// stencil cells from global memory (gather variant 3)
template <typename R> void launch_part_drag(const Desc &D, const Cells<R> &C, int record, hipStream_t s)
{
    if (D.pt.np == 0) return;
    if (D.t.gather == 3) {
        hipLaunchKernelGGL(k_part_drag<R>, dim3(nblocks(D.pt.np)), dim3(kBlock), 0, s, D, C, record);
        return;
    }
    // FP32: tiles of 16x8x8 cells (a halo of 1.76 cells per owned cell
    // against 2.1 for 16x4x8; 67 vs 71.5 us on the dilute workload); FP64
    // keeps 16x4x8, whose 7 staged fields stay within 64 KiB of LDS
    constexpr int TY = sizeof(R) == 4 ? 8 : 4;
    dim3 grid((D.g.n[0] + 15) / 16, (D.g.n[1] + TY - 1) / TY, (D.g.n[2] + 7) / 8);
    hipLaunchKernelGGL((k_part_tile<R, PASS_DRAG, 16, TY, 8>), grid, dim3(256), 0, s, D, C, record);
}
template <typename R> void launch_gather_fd(const Desc &D, const Cells<R> &C, hipStream_t s)
{
    launch_gather<R, MODE_FD>(D, C, s);
}
template <typename R> void launch_gather_eps(const Desc &D, const Cells<R> &C, hipStream_t s)
{
    launch_gather<R, MODE_EPS>(D, C, s);
}
template <typename R> void launch_gather_eps_uf(const Desc &D, const Cells<R> &C, hipStream_t s)
{
    launch_gather<R, MODE_EPS_UF>(D, C, s);
}
template <typename R> void launch_gather_eps_am(const Desc &D, const Cells<R> &C, hipStream_t s)
{
    launch_gather<R, MODE_EPS_AM>(D, C, s);
}
// The per-cell relaxation time (Eilers, LES) is a separate instance so that
// the constant-tau kernel keeps its code.
// Residency cap: the FP32 instances need few registers and would run 5 or 8
// waves per SIMD. Reserving 40,000 B of (unused) dynamic LDS per 256-thread
// workgroup limits a CU (160 KiB of LDS) to 4 workgroups, 4 waves per SIMD,
// which is fastest for this kernel's 38 PDF streams: on 256 x 256 x 512
// cells 8 waves/SIMD take 1.175 ms, 6 1.15 ms, 5 1.14 ms, 4 1.125 ms and
// 3 1.33 ms. The FP64 instances already run at 4 and 3 waves per SIMD.
template <typename R> void launch_stream_collide(const Desc &D, const Cells<R> &C, hipStream_t s)
{
    const unsigned lds = cell_lds_bytes(D.t.cell_waves, sizeof(R) == 4 ? 40000u : 0u);
    if (D.p.use_eilers || D.p.use_les)
        hipLaunchKernelGGL((k_stream_collide<R, true>), dim3(nblocks(D.g.nc)), dim3(kBlock), lds, s, D, C);
    else
        hipLaunchKernelGGL((k_stream_collide<R, false>), dim3(nblocks(D.g.nc)), dim3(kBlock), lds, s, D, C);
}
template <typename R> void launch_zero(R *p, int64_t n, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_zero<R>, dim3(grid_stride_blocks(n)), dim3(kBlock), 0, s, p, n);
}
template <typename R> void launch_fluid_fraction(const R *src, double *dst, int64_t nc, hipStream_t s)
{
    if (nc > 0)
        hipLaunchKernelGGL((k_fluid_fraction<R>), dim3(grid_stride_blocks(nc)), dim3(kBlock), 0, s, src, dst, nc);
}
template <typename R> void launch_vec4_to_double(const R *src, double *dst, int64_t nc, hipStream_t s)
{
    if (nc > 0)
        hipLaunchKernelGGL((k_vec4_to_soa<R>), dim3(grid_stride_blocks(nc)), dim3(kBlock), 0, s, src, dst, nc);
}
template <typename R> void launch_to_double(const R *src, double *dst, int64_t n, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL((k_convert<R, double>), dim3(grid_stride_blocks(n)), dim3(kBlock), 0, s, src, dst, n);
}
template <typename R> void launch_from_double(const double *src, R *dst, int64_t n, hipStream_t s)
{
    if (n > 0)
        hipLaunchKernelGGL((k_convert<double, R>), dim3(grid_stride_blocks(n)), dim3(kBlock), 0, s, src, dst, n);
}
int diag_blocks(const Desc &D)
{
    int64_t n = D.g.nc > D.pt.np ? D.g.nc : D.pt.np;
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b > kDiagMaxBlocks) b = kDiagMaxBlocks;
    return (int)(b < 1 ? 1 : b);
}

// Scratch of the allocation-free diagnostics (lbdem_diagnostics_noalloc):
// the per-block partials and the final values of k_diag / k_diag_final,
// 12 x 1024 + 16 doubles (98.4 KB), one copy per device for the life of the
// process. Host code never names the array itself (on the host it is only a
// stand-in): it uses the device address that hipGetSymbolAddress returns,
// looked up once per device with that device current.
static __device__ __align__(256) double scratch[kDiagScratchDoubles];

double *diag_scratch_on_device(int device)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess || cur != device) return nullptr;
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        addr[device] = static_cast<double *>(p);
    }
    return addr[device];
}
template <typename R>
void launch_diag(const Desc &D, const Cells<R> &C, const R *df, double *partials, int nblk, double *out,
                 hipStream_t s)
{
    hipLaunchKernelGGL(k_diag<R>, dim3(nblk), dim3(kBlock), 0, s, D, C, df, partials);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, s, (const double *)partials, nblk, out);
}

void launch_dem_force(const Desc &D, hipStream_t s)
{
    if (D.pt.np == 0) return;
    const dim3 g(nblocks(D.pt.np)), b(kBlock);
    const bool ns = use_nslot(D);
    if (D.pt.pk) {
        if (ns) hipLaunchKernelGGL((k_dem_force<double, true, true, false>), g, b, 0, s, D, 0, 0);
        else hipLaunchKernelGGL((k_dem_force<double, true, false, false>), g, b, 0, s, D, 0, 0);
    } else {
        if (ns) hipLaunchKernelGGL((k_dem_force<double, false, true, false>), g, b, 0, s, D, 0, 0);
        else hipLaunchKernelGGL((k_dem_force<double, false, false, false>), g, b, 0, s, D, 0, 0);
    }
}
bool dem_substep_fused(const Desc &D) { return D.pt.pk && use_nslot(D) && D.t.fuse == 1; }
void launch_dem_substep_fused(const Desc &D, int sub, int last, hipStream_t s)
{
    if (D.pt.np == 0) return;
    hipLaunchKernelGGL((k_dem_force<double, true, true, true>), dim3(nblocks(D.pt.np)), dim3(kBlock), 0, s, D, last,
                       sub & 1);
}
void launch_dem_order(const Desc &D, hipStream_t s)
{
    if (D.pt.np == 0 || !D.t.dem_order) return;
    const unsigned nb = nblocks(D.o.nrows, kScanPerBlock);
    hipLaunchKernelGGL(k_order_scan, dim3(nb), dim3(kBlock), 0, s, D);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, D.o.rowsum, (int)nb, D.o.rowsum + nb);
    hipLaunchKernelGGL(k_order_fill, dim3(nblocks(D.o.nrows)), dim3(kBlock), 0, s, D);
}
void launch_nlist(const Desc &D, hipStream_t s)
{
    if (D.pt.np <= 0) return;
    hipLaunchKernelGGL(k_nlist, dim3(nblocks(D.pt.np)), dim3(kBlock), 0, s, D);
    if (use_nslot(D))
        hipLaunchKernelGGL(k_nslot, dim3((unsigned)(((uint64_t)D.pt.np * kNslotLanes + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, s, D);
}
void launch_integrate(const Desc &D, int last, hipStream_t s)
{
    if (D.pt.np > 0) hipLaunchKernelGGL(k_integrate, dim3(nblocks(D.pt.np)), dim3(kBlock), 0, s, D, last);
}
void launch_bin_count(const Desc &D, hipStream_t s)
{
    if (D.pt.np > 0) hipLaunchKernelGGL(k_bin_count, dim3(nblocks(D.pt.np)), dim3(kBlock), 0, s, D);
}
void launch_bin_build(const Desc &D, hipStream_t s)
{
    const unsigned nb = nblocks(D.g.nc, kScanPerBlock);
    hipLaunchKernelGGL(k_scan_block, dim3(nb), dim3(kBlock), 0, s, D);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, D.b.bsum, (int)nb, D.b.start + D.g.nc);
    if (D.pt.np > 0) hipLaunchKernelGGL(k_place, dim3(nblocks(D.pt.np)), dim3(kBlock), 0, s, D);
}
void launch_sort_permute(const Desc &D, hipStream_t s)
{
    hipLaunchKernelGGL(k_cellsort, dim3(nblocks(D.g.nc)), dim3(kBlock), 0, s, D);
    if (D.pt.np > 0) hipLaunchKernelGGL(k_permute, dim3(nblocks(D.pt.np)), dim3(kBlock), 0, s, D);
}
template <typename R> void launch_sort_permute_am(const Desc &D, const Cells<R> &C, hipStream_t s)
{
    hipLaunchKernelGGL(k_cellsort, dim3(nblocks(D.g.nc)), dim3(kBlock), 0, s, D);
    if (D.pt.np > 0) hipLaunchKernelGGL(k_permute_am<R>, dim3(nblocks(D.pt.np)), dim3(kBlock), 0, s, D, C);
}
void launch_zero_int(int *p, int64_t n, hipStream_t s) { launch_zero<int>(p, n, s); }
void launch_set_int(int *p, int v, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, p, v);
}
void launch_set_step(long long *stepc, long long v, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_step, dim3(1), dim3(1), 0, s, stepc, v);
}

#define LBDEM_INST(R)                                                                                     \
    template void launch_moments<R>(const Desc &, const Cells<R> &, hipStream_t);                          \
    template void launch_cellfields<R>(const Desc &, const Cells<R> &, hipStream_t);                       \
    template void launch_curl<R>(const Desc &, const Cells<R> &, hipStream_t);                            \
    template void launch_sort_permute_am<R>(const Desc &, const Cells<R> &, hipStream_t);                 \
    template void launch_part_am<R>(const Desc &, const Cells<R> &, hipStream_t);                          \
    template void launch_gather_am<R>(const Desc &, const Cells<R> &, hipStream_t);                        \
    template void launch_part_drag<R>(const Desc &, const Cells<R> &, int, hipStream_t);                        \
    template void launch_gather_fd<R>(const Desc &, const Cells<R> &, hipStream_t);                        \
    template void launch_gather_eps<R>(const Desc &, const Cells<R> &, hipStream_t);                       \
    template void launch_gather_eps_am<R>(const Desc &, const Cells<R> &, hipStream_t);                    \
    template void launch_gather_eps_uf<R>(const Desc &, const Cells<R> &, hipStream_t);                    \
    template void launch_stream_collide<R>(const Desc &, const Cells<R> &, hipStream_t);                   \
    template void launch_zero<R>(R *, int64_t, hipStream_t);                                                \
    template void launch_to_double<R>(const R *, double *, int64_t, hipStream_t);                          \
    template void launch_vec4_to_double<R>(const R *, double *, int64_t, hipStream_t);                     \
    template void launch_fluid_fraction<R>(const R *, double *, int64_t, hipStream_t);                     \
    template void launch_from_double<R>(const double *, R *, int64_t, hipStream_t);                        \
    template void launch_diag<R>(const Desc &, const Cells<R> &, const R *, double *, int, double *, hipStream_t);

LBDEM_INST(float)
LBDEM_INST(double)

}  // namespace lbdem
