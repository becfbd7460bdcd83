// hosc_kernels.hpp -- gfx950 kernels of the HOSC time step (Punia & Ray, arXiv
// 2411.06563, Sec. 2) and of its diagnostics (Secs. 4.2, 4.3).
//
// Layouts in HBM
//   natural   : N^3 doubles, node (i,j,k) at i + N*(j + N*k)  (u, v, w, theta, p,
//               eta, E*, and their level n-1 copies).  x is the unit-stride axis.
//   colour    : the red-black split used by the implicit solves.  Node (i,j,k) has
//               colour c = (i+j+k) & 1 and lives in colour array c at
//               (k*N + j)*H + (i >> 1), H = (N+1)/2.  Inside one (j,k) row all nodes
//               of a colour share the parity of i, so a wavefront that updates a row
//               of one colour reads its x-neighbours at q and q +- 1 of the other
//               colour and its y/z neighbours at the same q of the rows j+-1, k+-1:
//               every access is unit-stride and no cache line carries unused nodes.
//
// Each implicit 7-point row is stored divided by its centre weight C: for the
// momentum system s/C and a_d/C (off-diagonal weights (s -+ a_d)/C towards x_d +- h),
// b/C; for the energy system a_d/C (s/C is a constant).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hosc {

struct Geo {
    int N;          // nodes per side
    int H;          // entries per colour row
    int Q;          // colour-row entries that can hold interior nodes
    int pad;
    double h, h2, inv2h, invh2;
    double invN;            // 1/N (node index arithmetic of the all-node launches)
    double h2_12, inv3h, inv12h, inv6h2;   // h^2/12, 1/(3h), 1/(12h), 1/(6h^2) (uniform grid: h = k = l)
    size_t n3;      // N^3
    size_t cs;      // entries of one colour array (N*N*H)
};

struct Phys {
    double Ra, Pr, dt, theta_hot, theta_cold, theta_ref, i2_floor, ex, lambda, phi;
};

__device__ __forceinline__ size_t nid(const Geo &g, int i, int j, int k)
{
    return (size_t)i + (size_t)g.N * ((size_t)j + (size_t)g.N * (size_t)k);
}
__device__ __forceinline__ size_t rowid(const Geo &g, int j, int k) { return ((size_t)k * g.N + j) * g.H; }

// ---------------------------------------------------------------------------
// Deterministic block reductions (fixed shuffle tree inside a wavefront, fixed
// order across the wavefronts of a block).  Every thread of the block must call.
// ---------------------------------------------------------------------------
template <int NV>
__device__ __forceinline__ void block_sum_store(double (&v)[NV], double *out, unsigned store = ~0u)
{
    __shared__ double sh[NV][16];
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthr = blockDim.x * blockDim.y * blockDim.z;
    const int lane = tid & 63, wave = tid >> 6, nwave = (nthr + 63) >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = v[q];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) sh[q][wave] = x;
    }
    __syncthreads();
    if (tid < NV && ((store >> tid) & 1u)) {
        double s = 0.0;
        for (int w = 0; w < nwave; ++w) s += sh[tid][w];
        out[tid] = s;
    }
}

// Block sums stored to up to two places, each with its own component mask.
template <int NV>
__device__ __forceinline__ void block_sum_store2(double (&v)[NV], double *out1, unsigned m1, double *out2, unsigned m2)
{
    __shared__ double sh[NV][16];
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthr = blockDim.x * blockDim.y * blockDim.z;
    const int lane = tid & 63, wave = tid >> 6, nwave = (nthr + 63) >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = v[q];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        if (lane == 0) sh[q][wave] = x;
    }
    __syncthreads();
    if (tid < NV) {
        double s = 0.0;
        for (int w = 0; w < nwave; ++w) s += sh[tid][w];
        if ((m1 >> tid) & 1u) out1[tid] = s;
        if ((m2 >> tid) & 1u) out2[tid] = s;
    }
}

// max that propagates NaN
__device__ __forceinline__ double nanmax(double a, double b) { return (a > b || a != a) ? a : b; }

template <int NV>
__device__ __forceinline__ void block_max_store(double (&v)[NV], double *out)
{
    __shared__ double sh[NV][16];
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthr = blockDim.x * blockDim.y * blockDim.z;
    const int lane = tid & 63, wave = tid >> 6, nwave = (nthr + 63) >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double x = v[q];
        for (int off = 32; off > 0; off >>= 1) x = nanmax(x, __shfl_down(x, off, 64));
        if (lane == 0) sh[q][wave] = x;
    }
    __syncthreads();
    if (tid < NV) {
        double s = sh[tid][0];
        for (int w = 1; w < nwave; ++w) s = nanmax(s, sh[tid][w]);
        out[tid] = s;
    }
}

// Reduce nb partial records of nc <= 8 values (record b at part[b*nc ...]) with one
// block of 1024 threads; op 0 = sum, 1 = max.  Thread t folds records t, t+1024, ...
// in order, then a fixed shuffle tree inside each wavefront and a fixed-order pass
// over the 16 wavefronts: deterministic.
// Thread t folds records t, t + 1024, ... of every component (the loads of four
// records issued together); per component the order is that of a
// component-by-component pass.
template <int NC>
__device__ __forceinline__ void fold_records(const double *part, int nb, int op, double (&acc)[8])
{
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = op == 0 ? 0.0 : -HUGE_VAL;
    // four records per pass, their loads issued together (a record past the end
    // reads the last record and is not folded), folded in the order b, b + 1024, ...
    for (int b = threadIdx.x; b < nb; b += 4096) {
        double x[4][NC];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int bb = min(b + 1024 * r, nb - 1);
#pragma unroll
            for (int c = 0; c < NC; ++c) x[r][c] = part[(size_t)bb * NC + c];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (b + 1024 * r >= nb) break;
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[c] = op == 0 ? acc[c] + x[r][c] : nanmax(acc[c], x[r][c]);
        }
    }
}

// A value written to pinned host memory (mapped, coherent) as well: a system-scope
// store and fence, so the host reads it once the stream has completed, without a
// device-to-host copy.
__device__ __forceinline__ void store_host(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __threadfence_system();
}

// out_host (may be null): the same outputs to mapped host memory.
__device__ __forceinline__ void reduce_block(const double *part, int nb, int nc, int op, double *out,
                                             double *out_host = nullptr)
{
    __shared__ double sh[8][16];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    double acc[8];
    switch (nc) {
    case 1: fold_records<1>(part, nb, op, acc); break;
    case 2: fold_records<2>(part, nb, op, acc); break;
    case 3: fold_records<3>(part, nb, op, acc); break;
    case 4: fold_records<4>(part, nb, op, acc); break;
    case 5: fold_records<5>(part, nb, op, acc); break;
    case 6: fold_records<6>(part, nb, op, acc); break;
    case 7: fold_records<7>(part, nb, op, acc); break;
    default: fold_records<8>(part, nb, op, acc); break;    // nc <= 8 (the size of sh)
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (c >= nc) break;
        double s = acc[c];
        for (int off = 32; off > 0; off >>= 1) {
            const double y = __shfl_down(s, off, 64);
            s = op == 0 ? s + y : nanmax(s, y);
        }
        if (lane == 0) sh[c][wave] = s;
    }
    __syncthreads();
    if (t < nc) {
        double s = sh[t][0];
        for (int w = 1; w < 16; ++w) s = op == 0 ? s + sh[t][w] : nanmax(s, sh[t][w]);
        out[t] = s;
        if (out_host) store_host(out_host + t, s);
    }
}

__global__ void __launch_bounds__(1024) k_reduce(const double *part, int nb, int nc, int op, double *out)
{
    reduce_block(part, nb, nc, op, out);
}

// Many reductions in one launch (one 1024-thread block per job), each computed
// exactly as k_reduce computes it.
struct ReduceJob {
    const double *part;
    double *out;
    double *out_host;       // null, or mapped host memory receiving the outputs too
    int nb, nc, op, pad;
};
__global__ void __launch_bounds__(1024) k_reduce_jobs(const ReduceJob *__restrict__ jobs)
{
    const ReduceJob jb = jobs[blockIdx.x];
    reduce_block(jb.part, jb.nb, jb.nc, jb.op, jb.out, jb.out_host);
}

// Up to four reductions passed by value (no table upload), one block each.
struct ReduceJobs4 {
    ReduceJob j[4];
};
__global__ void __launch_bounds__(1024) k_reduce4(ReduceJobs4 jobs)
{
    const ReduceJob &jb = jobs.j[blockIdx.x];
    reduce_block(jb.part, jb.nb, jb.nc, jb.op, jb.out, jb.out_host);
}

// Gather len doubles from each of gridDim.x device blocks into one contiguous array
// (one host copy then reads every cavity's reduction outputs).
// (dst: mapped host memory; the host reads it once the stream has completed.)
__global__ void __launch_bounds__(64) k_gather(const double *const *__restrict__ src, int len, double *__restrict__ dst)
{
    const double *s = src[blockIdx.x];
    for (int t = threadIdx.x; t < len; t += blockDim.x) store_host(dst + (size_t)blockIdx.x * len + t, s[t]);
}

// ---------------------------------------------------------------------------
// XCD-aware tile order.  Workgroups reach the eight XCDs round-robin by linear id;
// slot(b) hands each XCD a contiguous run of tiles (a balanced split of the G
// tiles into eight runs), so the rows and planes that neighbouring tiles share
// are read into the same L2.  Tile ids (and the partial-sum records indexed by them) are
// the plain linear order, so reductions see the same records in the same order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int persistent_slot(int b, int G)
{
    // G = 8q + r: XCD x (x = b mod 8) receives q + (x < r) workgroups and the
    // contiguous slots starting at x q + min(x, r)
    const int q = G >> 3, r = G & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

struct Tile {
    int x, y, z, id;
};
// Tile of block b of a launch of G = gx * gy * gz blocks (gx, gy: the grid's x and y
// extents), in the XCD-grouped order.
__device__ __forceinline__ Tile xcd_tile_of(int b, int G, int gx, int gy)
{
    Tile t;
    t.id = persistent_slot(b, G);
    t.x = t.id % gx;
    const int rest = t.id / gx;
    t.y = rest % gy;
    t.z = rest / gy;
    return t;
}
__device__ __forceinline__ Tile xcd_tile()
{
    const int G = gridDim.x * gridDim.y * gridDim.z;
    const int b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    return xcd_tile_of(b, G, gridDim.x, gridDim.y);
}

// Slab-ordered tiles of the interior launch (64 x 4 threads, one plane per tile
// row): the gy y-tiles are cut into eight slabs of ys = ceil(gy/8), one per XCD,
// and an XCD walks its slab plane after plane (x fastest, then y within the slab,
// then z), so the planes k-1, k, k+1 that a 19-point stencil reads are still in its
// L2 when the next plane needs them.  The launch is 1D with gx * ys * gz * 8
// workgroups; those past the last y-tile return at once (all their threads).  The
// tile id (and its partial-sum record) is the plain linear order.
__device__ __forceinline__ bool slab_tile(int gx, int gy, int gz, Tile &t)
{
    const int ys = (gy + 7) >> 3, per = gx * ys * gz;
    const int id = persistent_slot((int)blockIdx.x, 8 * per);
    const int slab = id / per, r = id - slab * per;
    t.x = r % gx;
    const int rest = r / gx;
    t.z = rest / ys;
    t.y = slab * ys + (rest - t.z * ys);
    t.id = t.x + gx * (t.y + gy * t.z);
    return t.y < gy;
}

// Node of a thread in a launch over every node: one thread per node in storage
// order (x fastest), 256-thread blocks of a 1D grid taken in XCD-grouped order, so
// no wave idles on the partial x-rows a 2D tiling leaves when N is not a multiple
// of 64.  False past the last node.  (n + 1/2)/N lies at least 1/(2N) from an
// integer, far above the FP64 rounding of the product, so the quotients are exact.
__device__ __forceinline__ bool all_node(const Geo &g, const Tile &tl, int &i, int &j, int &k)
{
    const int n = tl.id * (int)blockDim.x + (int)threadIdx.x;
    if ((size_t)n >= g.n3) return false;
    const int row = (int)(((double)n + 0.5) * g.invN);
    k = (int)(((double)row + 0.5) * g.invN);
    j = row - k * g.N;
    i = n - row * g.N;
    return true;
}

// ---------------------------------------------------------------------------
// Derivatives at any node: central inside, 2nd-order one-sided on a wall normal to
// the axis (velocity, eta, theta); the wall-normal pressure derivative is zero.
// Branch-free: every lane combines the node's own value fc (loaded once per field
// and shared by its three axes) with two more points at offsets and weights chosen
// per lane (inside: 0 fc + f(+1) - f(-1), exactly the central difference; on a wall
// the one-sided weights -3, 4, -1 on fc, f(+1), f(+2), or 3, -4, 1 on fc, f(-1),
// f(-2)), so the loads of all the derivatives of a node issue together instead of
// the wall and interior paths of a wavefront running one after the other (nearly
// every wavefront of an all-node launch holds an x-wall lane).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double dnode(const double *f, double fc, size_t c, size_t s, int idx, int N, double inv2h)
{
    const bool lo = idx == 0, hi = idx == N - 1;
    const ptrdiff_t t = (ptrdiff_t)s;
    const ptrdiff_t o1 = hi ? -t : t, o2 = lo ? 2 * t : (hi ? -2 * t : -t);
    const double w0 = lo ? -3.0 : (hi ? 3.0 : 0.0), w1 = lo ? 4.0 : (hi ? -4.0 : 1.0), w2 = lo ? -1.0 : (hi ? 1.0 : -1.0);
    const double b = f[(ptrdiff_t)c + o1], e = f[(ptrdiff_t)c + o2];
    return (w0 * fc + w1 * b + w2 * e) * inv2h;
}
__device__ __forceinline__ double dpnode(const double *p, size_t c, size_t s, int idx, int N, double inv2h)
{
    // on a wall both reads are the node itself: p - p = 0
    const ptrdiff_t o = (idx == 0 || idx == N - 1) ? 0 : (ptrdiff_t)s;
    return (p[(ptrdiff_t)c + o] - p[(ptrdiff_t)c - o]) * inv2h;
}

struct VelGrad {
    double ux, uy, uz, vx, vy, vz, wx, wy, wz;
};

__device__ __forceinline__ VelGrad vel_grad(const Geo &g, const double *u, const double *v, const double *w, int i,
                                            int j, int k)
{
    const size_t c = nid(g, i, j, k), sy = (size_t)g.N, sz = (size_t)g.N * g.N;
    const double uc = u[c], vc = v[c], wc = w[c];
    VelGrad d;
    d.ux = dnode(u, uc, c, 1, i, g.N, g.inv2h);
    d.uy = dnode(u, uc, c, sy, j, g.N, g.inv2h);
    d.uz = dnode(u, uc, c, sz, k, g.N, g.inv2h);
    d.vx = dnode(v, vc, c, 1, i, g.N, g.inv2h);
    d.vy = dnode(v, vc, c, sy, j, g.N, g.inv2h);
    d.vz = dnode(v, vc, c, sz, k, g.N, g.inv2h);
    d.wx = dnode(w, wc, c, 1, i, g.N, g.inv2h);
    d.wy = dnode(w, wc, c, sy, j, g.N, g.inv2h);
    d.wz = dnode(w, wc, c, sz, k, g.N, g.inv2h);
    return d;
}

// Second invariant of the strain rate (Sec. 2.1, viscosity formula).
__device__ __forceinline__ double strain_I2(const VelGrad &d)
{
    const double a = d.uz + d.wx, b = d.uy + d.vx, e = d.vz + d.wy;
    return 2.0 * (d.ux * d.ux + d.vy * d.vy + d.wz * d.wz) + a * a + b * b + e * e;
}

// eta = max(I2, floor)^((n-1)/2) at every node (Sec. 2.1, power law).
__global__ void __launch_bounds__(256) k_eta(Geo g, Phys P, const double *__restrict__ u, const double *__restrict__ v,
                                             const double *__restrict__ w, double *__restrict__ eta)
{
    const Tile tl = xcd_tile();
    int i, j, k;
    if (!all_node(g, tl, i, j, k)) return;
    const VelGrad d = vel_grad(g, u, v, w, i, j, k);
    eta[nid(g, i, j, k)] = pow(fmax(strain_I2(d), P.i2_floor), P.ex);
}

// Momentum sources at every node: the right-hand sides of the three momentum
// equations (Sec. 2.1, expanded stress divergence) divided by Pr eta, which puts
// them in the form of the generic transport PDE with L = 1/(Pr eta).
__global__ void __launch_bounds__(256) k_estar(Geo g, Phys P, const double *__restrict__ u,
                                               const double *__restrict__ v, const double *__restrict__ w,
                                               const double *__restrict__ T, const double *__restrict__ p,
                                               const double *__restrict__ eta, double *__restrict__ Eu,
                                               double *__restrict__ Ev, double *__restrict__ Ew)
{
    const Tile tl = xcd_tile();
    int i, j, k;
    if (!all_node(g, tl, i, j, k)) return;
    const size_t c = nid(g, i, j, k), sy = (size_t)g.N, sz = (size_t)g.N * g.N;
    const VelGrad d = vel_grad(g, u, v, w, i, j, k);
    const double etac = eta[c];
    const double ex = dnode(eta, etac, c, 1, i, g.N, g.inv2h), ey = dnode(eta, etac, c, sy, j, g.N, g.inv2h),
                 ez = dnode(eta, etac, c, sz, k, g.N, g.inv2h);
    const double px = dpnode(p, c, 1, i, g.N, g.inv2h), py = dpnode(p, c, sy, j, g.N, g.inv2h),
                 pz = dpnode(p, c, sz, k, g.N, g.inv2h);
    const double L = 1.0 / (P.Pr * etac);
    const double sxy = d.uy + d.vx, sxz = d.uz + d.wx, syz = d.vz + d.wy;
    Eu[c] = L * (-px + P.Pr * (2.0 * d.ux * ex + sxy * ey + sxz * ez));
    Ev[c] = L * (-py + P.Pr * (sxy * ex + 2.0 * d.vy * ey + syz * ez) + P.Ra * P.Pr * (T[c] - P.theta_ref));
    Ew[c] = L * (-pz + P.Pr * (sxz * ex + syz * ey + 2.0 * d.wz * ez));
}

// ---------------------------------------------------------------------------
// HOSC assembly at one interior node (Sec. 2.2).
//
// Implicit side: the seven weights L1..L7 of the paper, written as
//     L1, L2 = s -+ a_x,  L3, L4 = s -+ a_y,  L5, L6 = s -+ a_z,  L7 = C
// with c = L M_1 (= L h^2/12 - dt/2), s = c/h^2, e_d = L M15 (= (h^2/6) delta_d L),
// a_d = (c V_d - e_d)/(2h), C = L (1 + 2 M_4 M18/dt) - 6 c/h^2.
// Explicit side: b = sum_m Q_m chi_m + dt R - sum_m L_m chi_m, i.e. the paper's Q
// weights minus the L weights: on the 7 central points Q - L keeps the dt alpha,
// dt M1, ... parts of N1..N6; on the 12 edge points Q is taken as printed.  We
// store W_m = (Q_m - L_m)/dt and form b = dt (R + sum_m W_m chi_m).
// ---------------------------------------------------------------------------

// Offsets of the 19 points in the paper's Q numbering: centre, x+, x-, y+, y-, z+, z-
// (Q2, Q1, Q3, Q4, Q5, Q6, Q7), then Q8..Q19.
struct Coef19 {
    double W[19];
};

// W_m = (Q_m - L_m)/dt for a system with convection V = (G, H, I) given at the 7
// central points (index 0 centre, 1 x+, 2 x-, 3 y+, 4 y-, 5 z+, 6 z-) and at level
// n-1 at the centre.
__device__ __forceinline__ void explicit_weights(const Geo &g, double dt, const double (&G)[7], const double (&Hc)[7],
                                                 const double (&I)[7], double Gp, double Hp, double Ip, Coef19 &cw)
{
    // On the uniform grid (h = k = l) the grid factors of the expanded weights
    // reduce to constants: M5 = M6 = M7 = h^2/6, M5/(h^2 k^2) = 1/(6h^2),
    // M5/(h k^2) = 1/(6h) (twice per weight: 1/(3h)), M5/(4hk) = 1/24,
    // M5/(2 h k^2) = 1/(12h), and 2/(h^2 + k^2) (k^2 a + h^2 b) = a + b; the
    // (dt/2) delta_t^- terms are (f^n - f^(n-1))/2.  Products with precomputed
    // reciprocals replace the divisions of the printed form.
    (void)dt;
    const double i2h = g.inv2h, ih2 = g.invh2, h12 = g.h2_12;
    const double G0 = G[0], H0 = Hc[0], I0 = I[0];
    // first and second central differences of the convective coefficients
    const double Gx = (G[1] - G[2]) * i2h, Gy = (G[3] - G[4]) * i2h, Gz = (G[5] - G[6]) * i2h;
    const double Hx = (Hc[1] - Hc[2]) * i2h, Hy = (Hc[3] - Hc[4]) * i2h, Hz = (Hc[5] - Hc[6]) * i2h;
    const double Ix = (I[1] - I[2]) * i2h, Iy = (I[3] - I[4]) * i2h, Iz = (I[5] - I[6]) * i2h;
    const double Gxx = (G[1] - 2.0 * G0 + G[2]) * ih2, Gyy = (G[3] - 2.0 * G0 + G[4]) * ih2,
                 Gzz = (G[5] - 2.0 * G0 + G[6]) * ih2;
    const double Hxx = (Hc[1] - 2.0 * H0 + Hc[2]) * ih2, Hyy = (Hc[3] - 2.0 * H0 + Hc[4]) * ih2,
                 Hzz = (Hc[5] - 2.0 * H0 + Hc[6]) * ih2;
    const double Ixx = (I[1] - 2.0 * I0 + I[2]) * ih2, Iyy = (I[3] - 2.0 * I0 + I[4]) * ih2,
                 Izz = (I[5] - 2.0 * I0 + I[6]) * ih2;
    // alpha, beta, gamma (K* = 0)
    const double alpha = (G0 * G0 - 2.0 * Gx) * h12 + 1.0;
    const double beta = (H0 * H0 - 2.0 * Hy) * h12 + 1.0;
    const double gamma = (I0 * I0 - 2.0 * Iz) * h12 + 1.0;
    // M1, M2, M3: the bracket [1 + (dxx - G dx) h^2/12 + (dyy - H dy) k^2/12 +
    // (dzz - I dz) l^2/12 + (dt/2) delta_t^-] applied to G*, H*, I*
    const double M1 = G0 + ((Gxx - G0 * Gx) + (Gyy - H0 * Gy) + (Gzz - I0 * Gz)) * h12 + 0.5 * (G0 - Gp);
    const double M2 = H0 + ((Hxx - G0 * Hx) + (Hyy - H0 * Hy) + (Hzz - I0 * Hz)) * h12 + 0.5 * (H0 - Hp);
    const double M3 = I0 + ((Ixx - G0 * Ix) + (Iyy - H0 * Iy) + (Izz - I0 * Iz)) * h12 + 0.5 * (I0 - Ip);
    const double p1 = -G0 * H0 + (Gy + Hx);
    const double q1 = -H0 * I0 + (Hz + Iy);
    const double r1 = -I0 * G0 + (Ix + Gz);
    const double c = g.inv6h2, c4 = 4.0 * c, i3h = g.inv3h, i12h = g.inv12h;
    // Q2 - L7 and Q1 - L1 ... Q7 - L6, divided by dt
    cw.W[0] = -2.0 * (alpha + beta + gamma) * ih2 + 12.0 * c;
    cw.W[1] = alpha * ih2 - M1 * i2h - c4 + G0 * i3h;
    cw.W[2] = alpha * ih2 + M1 * i2h - c4 - G0 * i3h;
    cw.W[3] = beta * ih2 - M2 * i2h - c4 + H0 * i3h;
    cw.W[4] = beta * ih2 + M2 * i2h - c4 - H0 * i3h;
    cw.W[5] = gamma * ih2 - M3 * i2h - c4 + I0 * i3h;
    cw.W[6] = gamma * ih2 + M3 * i2h - c4 - I0 * i3h;
    // Q8..Q19 / dt
    const double a5 = p1 * (1.0 / 24.0), g5 = G0 * i12h, h5 = H0 * i12h;
    cw.W[7] = c - a5 - h5 - g5;     // (i+1, j+1)
    cw.W[8] = c + a5 - h5 + g5;     // (i-1, j+1)
    cw.W[9] = c + a5 + h5 - g5;     // (i+1, j-1)
    cw.W[10] = c - a5 + h5 + g5;    // (i-1, j-1)
    const double a6 = q1 * (1.0 / 24.0), i6 = I0 * i12h, h6 = H0 * i12h;
    cw.W[11] = c - a6 - i6 - h6;    // (j+1, k+1)
    cw.W[12] = c + a6 - i6 + h6;    // (j-1, k+1)
    cw.W[13] = c + a6 + i6 - h6;    // (j+1, k-1)
    cw.W[14] = c - a6 + i6 + h6;    // (j-1, k-1)
    const double a7 = r1 * (1.0 / 24.0), g7 = G0 * i12h, i7 = I0 * i12h;
    cw.W[15] = c - a7 - g7 - i7;    // (i+1, k+1)
    cw.W[16] = c + a7 - g7 + i7;    // (i+1, k-1)
    cw.W[17] = c + a7 + g7 - i7;    // (i-1, k+1)
    cw.W[18] = c - a7 + g7 + i7;    // (i-1, k-1)
}

__device__ __forceinline__ void offsets19(const Geo &g, size_t c, size_t (&o)[19])
{
    const size_t sy = (size_t)g.N, sz = (size_t)g.N * g.N;
    o[0] = c;
    o[1] = c + 1; o[2] = c - 1; o[3] = c + sy; o[4] = c - sy; o[5] = c + sz; o[6] = c - sz;
    o[7] = c + 1 + sy; o[8] = c - 1 + sy; o[9] = c + 1 - sy; o[10] = c - 1 - sy;
    o[11] = c + sy + sz; o[12] = c - sy + sz; o[13] = c + sy - sz; o[14] = c - sy - sz;
    o[15] = c + 1 + sz; o[16] = c + 1 - sz; o[17] = c - 1 + sz; o[18] = c - 1 - sz;
}

// bracket operator of the source: R = [1 + sum (d_dd - V_d d_d) h^2/12 + (dt/2) delta_t^-] E*
__device__ __forceinline__ double source_R(const Geo &g, double dt, const double (&E)[7], double Ep, double G0,
                                           double H0, double I0)
{
    (void)dt;   // (dt/2) delta_t^- E = (E^n - E^(n-1))/2
    const double Ex = (E[1] - E[2]) * g.inv2h, Ey = (E[3] - E[4]) * g.inv2h, Ez = (E[5] - E[6]) * g.inv2h;
    const double Exx = (E[1] - 2.0 * E[0] + E[2]) * g.invh2, Eyy = (E[3] - 2.0 * E[0] + E[4]) * g.invh2,
                 Ezz = (E[5] - 2.0 * E[0] + E[6]) * g.invh2;
    return E[0] + ((Exx - G0 * Ex) + (Eyy - H0 * Ey) + (Ezz - I0 * Ez)) * g.h2_12 + 0.5 * (E[0] - Ep);
}

struct NodeAssembly {
    double Cm, sm, am[3];   // momentum row: centre, s, a_d
    double Ct, st, at[3];   // energy row
    double b[4];            // right-hand sides of the u, v, w, theta increments
};

// Implicit 7-point row of the generic PDE (Eq. 1, K* = 0) at an interior node, from
// L at the 7 central points (level n), the convective coefficients at the centre and
// L at the centre at level n-1: centre C and the weights s -+ a_d towards x_d +- h.
__device__ __forceinline__ void implicit_row(const Geo &g, double dt, const double (&Lm)[7], double G0, double H0,
                                             double I0, double Lp, double &C, double &s, double (&a)[3])
{
    const double L0 = Lm[0];
    const double Lx = (Lm[1] - Lm[2]) * g.inv2h, Ly = (Lm[3] - Lm[4]) * g.inv2h, Lz = (Lm[5] - Lm[6]) * g.inv2h;
    const double Lxx = (Lm[1] - 2.0 * L0 + Lm[2]) * g.invh2, Lyy = (Lm[3] - 2.0 * L0 + Lm[4]) * g.invh2,
                 Lzz = (Lm[5] - 2.0 * L0 + Lm[6]) * g.invh2;
    // M18 = [(dt/2) delta_t^- + sum (d_dd - V_d d_d) h_d^2/12] L
    const double M18 = 0.5 * (L0 - Lp) + ((Lxx - G0 * Lx) + (Lyy - H0 * Ly) + (Lzz - I0 * Lz)) * g.h2_12;
    // c = L M_1 = L h^2/12 - dt/2 (M_1 = M_2 = M_3 for h = k = l); the centre
    // (1 + 2 M_4 M18 / dt) L with M_4 = dt/(2L) is L + M18
    const double cc = L0 * g.h2_12 - 0.5 * dt;
    C = L0 + M18 - 6.0 * cc * g.invh2;
    s = cc * g.invh2;
    // L M15 = (h^2/6) dL/dx, etc.
    a[0] = (cc * G0 - 2.0 * g.h2_12 * Lx) * g.inv2h;
    a[1] = (cc * H0 - 2.0 * g.h2_12 * Ly) * g.inv2h;
    a[2] = (cc * I0 - 2.0 * g.h2_12 * Lz) * g.inv2h;
}

template <typename Tin>
__device__ __forceinline__ void assemble_node(const Geo &g, const Phys &P, int i, int j, int k, const Tin *u,
                                              const Tin *v, const Tin *w, const Tin *T, const Tin *eta,
                                              const Tin *Eu, const Tin *Ev, const Tin *Ew, const Tin *up,
                                              const Tin *vp, const Tin *wp, const Tin *etap, const Tin *Eup,
                                              const Tin *Evp, const Tin *Ewp, NodeAssembly &out)
{
    const size_t c = nid(g, i, j, k);
    size_t o[19];
    offsets19(g, c, o);
    const double dt = P.dt;
    // ---- momentum coefficients: L = 1/(Pr eta), (G*, H*, I*) = (u, v, w) L
    double Lm[7], G[7], Hm[7], I[7];
#pragma unroll
    for (int m = 0; m < 7; ++m) {
        Lm[m] = 1.0 / (P.Pr * eta[o[m]]);
        G[m] = u[o[m]] * Lm[m];
        Hm[m] = v[o[m]] * Lm[m];
        I[m] = w[o[m]] * Lm[m];
    }
    const double Lp = 1.0 / (P.Pr * etap[c]);
    const double Gp = up[c] * Lp, Hp = vp[c] * Lp, Ip = wp[c] * Lp;
    implicit_row(g, dt, Lm, G[0], Hm[0], I[0], Lp, out.Cm, out.sm, out.am);
    // ---- momentum right-hand sides
    {
        Coef19 cw;
        explicit_weights(g, dt, G, Hm, I, Gp, Hp, Ip, cw);
        double su = 0.0, sv = 0.0, sw = 0.0;
#pragma unroll
        for (int m = 0; m < 19; ++m) {
            su += cw.W[m] * u[o[m]];
            sv += cw.W[m] * v[o[m]];
            sw += cw.W[m] * w[o[m]];
        }
        double E7[7];
#pragma unroll
        for (int m = 0; m < 7; ++m) E7[m] = Eu[o[m]];
        const double Ru = source_R(g, dt, E7, Eup[c], G[0], Hm[0], I[0]);
#pragma unroll
        for (int m = 0; m < 7; ++m) E7[m] = Ev[o[m]];
        const double Rv = source_R(g, dt, E7, Evp[c], G[0], Hm[0], I[0]);
#pragma unroll
        for (int m = 0; m < 7; ++m) E7[m] = Ew[o[m]];
        const double Rw = source_R(g, dt, E7, Ewp[c], G[0], Hm[0], I[0]);
        out.b[0] = dt * (Ru + su);
        out.b[1] = dt * (Rv + sv);
        out.b[2] = dt * (Rw + sw);
    }
    // ---- energy: L = 1, (G*, H*, I*) = (u, v, w), K* = E* = 0
    {
        double uu[7], vv[7], ww[7];
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            uu[m] = u[o[m]];
            vv[m] = v[o[m]];
            ww[m] = w[o[m]];
        }
        const double ct = g.h2_12 - 0.5 * dt;       // L M_1 with L = 1
        out.Ct = 1.0 - 6.0 * ct * g.invh2;          // M18 = 0 and M15..M17 = 0 for constant L
        out.st = ct * g.invh2;
        out.at[0] = ct * uu[0] * g.inv2h;
        out.at[1] = ct * vv[0] * g.inv2h;
        out.at[2] = ct * ww[0] * g.inv2h;
        Coef19 cw;
        explicit_weights(g, dt, uu, vv, ww, up[c], vp[c], wp[c], cw);
        double st = 0.0;
#pragma unroll
        for (int m = 0; m < 19; ++m) st += cw.W[m] * T[o[m]];
        out.b[3] = dt * st;
    }
}

struct ColourArrays {
    double *ms, *ma[3];             // momentum rows: s/C, a_d/C
    double *mb[3];                  // momentum right-hand sides b/C (u, v, w)
    double *ta[3];                  // energy rows: a_d/C
    double *tb;                     // energy right-hand side b/C
};

// Assemble every interior node and write the scaled rows in the colour layout;
// per-block partial sums of ||b/C||^2 for the four systems and the largest
// off-diagonal/centre ratio.  (The precision mode's FP32 copies come from a
// separate streaming pass: stores here would push the kernel past the register
// budget of two waves per SIMD.)
__global__ void __launch_bounds__(256) k_assemble(Geo g, Phys P, const double *__restrict__ u,
                                                  const double *__restrict__ v, const double *__restrict__ w,
                                                  const double *__restrict__ T, const double *__restrict__ eta,
                                                  const double *__restrict__ Eu, const double *__restrict__ Ev,
                                                  const double *__restrict__ Ew, const double *__restrict__ up,
                                                  const double *__restrict__ vp, const double *__restrict__ wp,
                                                  const double *__restrict__ etap, const double *__restrict__ Eup,
                                                  const double *__restrict__ Evp, const double *__restrict__ Ewp,
                                                  ColourArrays ca, double *__restrict__ partial,
                                                  double *__restrict__ partial_dom)
{
    const int M = g.N - 2;
    Tile tl;
    if (!slab_tile((M + 63) >> 6, (M + 3) >> 2, M, tl)) return;
    const int i = 1 + tl.x * blockDim.x + threadIdx.x, j = 1 + tl.y * blockDim.y + threadIdx.y, k = 1 + tl.z;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    double dom[2] = {0.0, 0.0};     // off-diagonal sum / |centre| of the momentum and energy rows
    if (i <= g.N - 2 && j <= g.N - 2) {
        NodeAssembly a;
        assemble_node(g, P, i, j, k, u, v, w, T, eta, Eu, Ev, Ew, up, vp, wp, etap, Eup, Evp, Ewp, a);
        const size_t idx = (size_t)((i + j + k) & 1) * g.cs + rowid(g, j, k) + (i >> 1);
        const double rm = 1.0 / a.Cm, rt = 1.0 / a.Ct;
        ca.ms[idx] = a.sm * rm;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            ca.ma[d][idx] = a.am[d] * rm;
            ca.ta[d][idx] = a.at[d] * rt;
            const double bb = a.b[d] * rm;
            ca.mb[d][idx] = bb;
            acc[d] = bb * bb;
        }
        const double bt = a.b[3] * rt;
        ca.tb[idx] = bt;
        acc[3] = bt * bt;
        double om = 0.0, ot = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            om += fabs(a.sm - a.am[d]) + fabs(a.sm + a.am[d]);
            ot += fabs(a.st - a.at[d]) + fabs(a.st + a.at[d]);
        }
        dom[0] = om / fabs(a.Cm);
        dom[1] = ot / fabs(a.Ct);
    }
    const int blk = tl.id;
    block_sum_store<4>(acc, partial + (size_t)blk * 4);
    block_max_store<2>(dom, partial_dom + (size_t)blk * 2);
}

// Parity hook: one selected assembled quantity, unscaled, in the natural layout:
// what 0..6 momentum weight (centre, x+, x-, y+, y-, z+, z-), 7..13 energy weight,

// FP32 copies of the scaled rows (precision mode): the seven row arrays of both
// colours, converted with round-to-nearest.
__global__ void __launch_bounds__(256) k_rows_f32(size_t n, const double *__restrict__ ms,
                                                  const double *__restrict__ mx, const double *__restrict__ my,
                                                  const double *__restrict__ mz, const double *__restrict__ tx,
                                                  const double *__restrict__ ty, const double *__restrict__ tz,
                                                  float *__restrict__ fms, float *__restrict__ fmx,
                                                  float *__restrict__ fmy, float *__restrict__ fmz,
                                                  float *__restrict__ ftx, float *__restrict__ fty,
                                                  float *__restrict__ ftz)
{
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x) {
        fms[q] = (float)ms[q];
        fmx[q] = (float)mx[q];
        fmy[q] = (float)my[q];
        fmz[q] = (float)mz[q];
        ftx[q] = (float)tx[q];
        fty[q] = (float)ty[q];
        ftz[q] = (float)tz[q];
    }
}

// 14..17 b of u, v, w, theta.
__global__ void __launch_bounds__(256) k_assemble_debug(Geo g, Phys P, const double *u, const double *v,
                                                        const double *w, const double *T, const double *eta,
                                                        const double *Eu, const double *Ev, const double *Ew,
                                                        const double *up, const double *vp, const double *wp,
                                                        const double *etap, const double *Eup, const double *Evp,
                                                        const double *Ewp, int what, double *out)
{
    const Tile tl = xcd_tile();
    const int i = 1 + tl.x * blockDim.x + threadIdx.x, j = 1 + tl.y * blockDim.y + threadIdx.y, k = 1 + tl.z;
    if (i > g.N - 2 || j > g.N - 2) return;
    NodeAssembly a;
    assemble_node(g, P, i, j, k, u, v, w, T, eta, Eu, Ev, Ew, up, vp, wp, etap, Eup, Evp, Ewp, a);
    double val;
    if (what < 14) {
        const bool mom = what < 7;
        const int m = what % 7;
        const double C = mom ? a.Cm : a.Ct, s = mom ? a.sm : a.st;
        const double *ad = mom ? a.am : a.at;
        if (m == 0) val = C;
        else {
            const int d = (m - 1) >> 1;
            val = (m & 1) ? s - ad[d] : s + ad[d];
        }
    } else {
        val = a.b[what - 14];
    }
    out[nid(g, i, j, k)] = val;
}

// ---------------------------------------------------------------------------
// One step of the generic transport PDE (Eq. 1, K* = 0) with coefficient fields
// given at every node (L, G*, H*, I*, E* at level n; at level n-1 only their centre
// values enter, through the time differences) and Dirichlet walls.  The row and b
// of each interior node are those of the momentum assembly with L and V read
// instead of formed from eta and the velocity; the known wall increments
// chi_new - chi of the six neighbours are moved to the right-hand side.  The scaled
// row goes to the first momentum system (the other two get b = 0, so their sweeps
// are skipped).  E and Ep may be null (zero source).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_assemble_transport(
    Geo g, double dt, const double *__restrict__ L, const double *__restrict__ G, const double *__restrict__ H,
    const double *__restrict__ I, const double *__restrict__ E, const double *__restrict__ Lp,
    const double *__restrict__ Gp, const double *__restrict__ Hp, const double *__restrict__ Ip,
    const double *__restrict__ Ep, const double *__restrict__ chi, const double *__restrict__ chi_new,
    ColourArrays ca, double *__restrict__ partial, double *__restrict__ partial_dom)
{
    const Tile tl = xcd_tile();
    const int i = 1 + tl.x * blockDim.x + threadIdx.x, j = 1 + tl.y * blockDim.y + threadIdx.y, k = 1 + tl.z;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    double dom[2] = {0.0, 0.0};
    if (i <= g.N - 2 && j <= g.N - 2) {
        const size_t c = nid(g, i, j, k);
        size_t o[19];
        offsets19(g, c, o);
        double Lm[7], Gv[7], Hv[7], Iv[7];
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            Lm[m] = L[o[m]];
            Gv[m] = G[o[m]];
            Hv[m] = H[o[m]];
            Iv[m] = I[o[m]];
        }
        double C, sw, a[3];
        implicit_row(g, dt, Lm, Gv[0], Hv[0], Iv[0], Lp[c], C, sw, a);
        Coef19 cw;
        explicit_weights(g, dt, Gv, Hv, Iv, Gp[c], Hp[c], Ip[c], cw);
        double sum = 0.0;
#pragma unroll
        for (int m = 0; m < 19; ++m) sum += cw.W[m] * chi[o[m]];
        double R = 0.0;
        if (E) {
            double E7[7];
#pragma unroll
            for (int m = 0; m < 7; ++m) E7[m] = E[o[m]];
            R = source_R(g, dt, E7, Ep[c], Gv[0], Hv[0], Iv[0]);
        }
        double b = dt * (R + sum);
        // neighbours 1..6 (x+, x-, y+, y-, z+, z-) with weights s - a_d, s + a_d
        const bool wall[6] = {i == g.N - 2, i == 1, j == g.N - 2, j == 1, k == g.N - 2, k == 1};
#pragma unroll
        for (int m = 0; m < 6; ++m)
            if (wall[m]) {
                const double wgt = (m & 1) ? sw + a[m >> 1] : sw - a[m >> 1];
                b -= wgt * (chi_new[o[m + 1]] - chi[o[m + 1]]);
            }
        const size_t idx = (size_t)((i + j + k) & 1) * g.cs + rowid(g, j, k) + (i >> 1);
        const double rc = 1.0 / C;
        ca.ms[idx] = sw * rc;
        double om = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            ca.ma[d][idx] = a[d] * rc;
            om += fabs(sw - a[d]) + fabs(sw + a[d]);
        }
        const double bb = b * rc;
        ca.mb[0][idx] = bb;
        ca.mb[1][idx] = 0.0;
        ca.mb[2][idx] = 0.0;
        acc[0] = bb * bb;
        dom[0] = om / fabs(C);
    }
    const int blk = tl.id;
    block_sum_store<4>(acc, partial + (size_t)blk * 4);
    block_max_store<2>(dom, partial_dom + (size_t)blk * 2);
}

// chi_new = chi + increment at interior nodes (walls of chi_new untouched).
__global__ void __launch_bounds__(256) k_transport_update(Geo g, const double *__restrict__ chi,
                                                          const double *__restrict__ d, double *__restrict__ chi_new)
{
    const Tile tl = xcd_tile();
    const int i = 1 + tl.x * blockDim.x + threadIdx.x, j = 1 + tl.y * blockDim.y + threadIdx.y, k = 1 + tl.z;
    if (i > g.N - 2 || j > g.N - 2) return;
    const size_t c = nid(g, i, j, k);
    chi_new[c] = chi[c] + d[(size_t)((i + j + k) & 1) * g.cs + rowid(g, j, k) + (i >> 1)];
}

// ---------------------------------------------------------------------------
// Scaled implicit rows in the colour layout.
//
// Momentum row at a node: d_c + sum_d [(s - a_d) d(x_d + h) + (s + a_d) d(x_d - h)] = b
// (everything divided by the centre weight; walls hold zero increments).
// Energy row: the same with s = st constant; next to a y or z wall the wall
// increment is (4 d_1 - d_2)/3, which moves 4/3 of the wall weight onto the centre
// (den) and -1/3 of it onto the next node.
// ---------------------------------------------------------------------------
struct RowIdx {
    size_t me, xp, xm, yp, ym, zp, zm;
};

__device__ __forceinline__ bool row_index(const Geo &g, int colour, int q, int j, int k, RowIdx &r)
{
    const int N = g.N;
    const int i = 2 * q + ((colour + j + k) & 1);
    if (q >= g.Q || j > N - 2 || k > N - 2 || i < 1 || i > N - 2) return false;
    const size_t row = rowid(g, j, k);
    const size_t ob = (size_t)(1 - colour) * g.cs;
    const int sh = i & 1;
    r.me = (size_t)colour * g.cs + row + q;
    r.xp = ob + row + q + sh;
    r.xm = ob + row + q + sh - 1;
    r.yp = ob + rowid(g, j + 1, k) + q;
    r.ym = ob + rowid(g, j - 1, k) + q;
    r.zp = ob + rowid(g, j, k + 1) + q;
    r.zm = ob + rowid(g, j, k - 1) + q;
    return true;
}

// off-diagonal sum of a momentum row for the vector given by f(index)
template <typename TA, typename F>
__device__ __forceinline__ TA mom_off(TA s, TA ax, TA ay, TA az, const RowIdx &r, F f)
{
    return (s - ax) * f(r.xp) + (s + ax) * f(r.xm) + (s - ay) * f(r.yp) + (s + ay) * f(r.ym) + (s - az) * f(r.zp)
           + (s + az) * f(r.zm);
}

// off-diagonal sum and centre factor of an energy row (walls eliminated)
template <typename TA, typename F>
__device__ __forceinline__ TA theta_off(TA st, TA ax, TA ay, TA az, int j, int k, int N, const RowIdx &r, F f, TA &den)
{
    const TA wxp = st - ax, wxm = st + ax, wyp = st - ay, wym = st + ay, wzp = st - az, wzm = st + az;
    const TA third = (TA)(1.0 / 3.0), four3 = (TA)(4.0 / 3.0);
    den = (TA)1.0;
    TA sum = wxp * f(r.xp) + wxm * f(r.xm);
    if (j == 1) {
        den += four3 * wym;
        sum += (wyp - wym * third) * f(r.yp);
    } else if (j == N - 2) {
        den += four3 * wyp;
        sum += (wym - wyp * third) * f(r.ym);
    } else {
        sum += wyp * f(r.yp) + wym * f(r.ym);
    }
    if (k == 1) {
        den += four3 * wzm;
        sum += (wzp - wzm * third) * f(r.zp);
    } else if (k == N - 2) {
        den += four3 * wzp;
        sum += (wzm - wzp * third) * f(r.zm);
    } else {
        sum += wzp * f(r.zp) + wzm * f(r.zm);
    }
    return sum;
}

// ---------------------------------------------------------------------------
// Red-black SOR half-sweep on the scaled rows (momentum: three right-hand sides
// on one matrix; energy with the walls eliminated).  Per-block partial sums of
// the squared scaled residuals r = b - B d at the updated nodes, before their
// update, are stored for the systems in `store` (bit f = system f) to `partial`, and
// for the systems in `store0` to `partial0` (the first sweep of a batch).
// ---------------------------------------------------------------------------
template <typename TM>
struct SweepArgs {
    const TM *ms, *ma[3], *mb[3];
    TM *md[3];
    const TM *ta[3], *tb;
    TM *td;
};

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

// Two consecutive entries of a colour array, 2 x sizeof(T) bytes at an even index
// (colour rows have an even length, so such a pair is aligned to its size).
template <typename T>
__device__ __forceinline__ typename Vec2<T>::type ld_pair(const T *x, size_t o)
{
    return *reinterpret_cast<const typename Vec2<T>::type *>(x + o);
}
template <typename T>
__device__ __forceinline__ void st_pair(T *x, size_t o, T a, T b)
{
    typename Vec2<T>::type v;
    v.x = a;
    v.y = b;
    *reinterpret_cast<typename Vec2<T>::type *>(x + o) = v;
}

// The other colour's values around the colour-row entries q0, q0 + 1 (par =
// (colour + j + k) & 1): the x neighbours (x- of entry 0, the shared one, x+ of
// entry 1) as one pair and one single value at xb = other colour's row + q0, then
// the y+, y-, z+, z- pairs; n0 / n1 in the neighbour order of mom_off / theta_off
// (0 x+, 1 x-, 2 y+, 3 y-, 4 z+, 5 z-).
template <typename T, typename TA>
__device__ __forceinline__ void pair_around(const T *d, int par, size_t xb, size_t yp, size_t ym, size_t zp, size_t zm,
                                            TA (&n0)[6], TA (&n1)[6])
{
    TA xlo, xmid, xhi;
    if (par) {
        const auto t = ld_pair(d, xb);
        xlo = (TA)t.x;
        xmid = (TA)t.y;
        xhi = (TA)d[xb + 2];
    } else {
        xlo = (TA)d[xb - 1];
        const auto t = ld_pair(d, xb);
        xmid = (TA)t.x;
        xhi = (TA)t.y;
    }
    const auto y1 = ld_pair(d, yp), y0 = ld_pair(d, ym), z1 = ld_pair(d, zp), z0 = ld_pair(d, zm);
    n0[0] = xmid; n0[1] = xlo; n0[2] = (TA)y1.x; n0[3] = (TA)y0.x; n0[4] = (TA)z1.x; n0[5] = (TA)z0.x;
    n1[0] = xhi; n1[1] = xmid; n1[2] = (TA)y1.y; n1[3] = (TA)y0.y; n1[4] = (TA)z1.y; n1[5] = (TA)z0.y;
}

// neighbour codes of mom_off / theta_off for values held in n0 / n1
__device__ __forceinline__ RowIdx pair_codes()
{
    RowIdx code;
    code.me = 6;
    code.xp = 0;
    code.xm = 1;
    code.yp = 2;
    code.ym = 3;
    code.zp = 4;
    code.zm = 5;
    return code;
}

// SOR updates of the two nodes at colour-row entries q0 = 2p and q0 + 1 of row
// (j, k) (nodes i = 2q + par, par = (colour + j + k) & 1), with loads of both
// entries at once: own-colour rows, right-hand sides and increments as pairs, the
// y and z neighbours as pairs of the other colour's rows, the three x neighbours
// (q0 + par - 1 .. q0 + par + 1) as one pair and one single value.  Each node's
// update is the same expression, in the same order, as for a node on its own.
// The squared pre-update residuals of both nodes go to r2.  mask: bit 0 momentum,
// bit 1 energy, bits 2..4 momentum fields u, v, w to leave alone (a zero
// right-hand side: zero increment), bit 5 the first sweep of a solve that starts
// from the zero increment (the stored values are not read: the colour-0 half
// takes its own and its neighbours' as zero, the colour-1 half its own).  An entry
// that holds no interior node keeps its stored value.
template <typename TM, typename TA>
__device__ __forceinline__ void sweep_pair(const Geo &g, int colour, int mask, TA omega_m, TA omega_t, TA st,
                                           const SweepArgs<TM> &a, int p, int j, int k, double (&r2)[4])
{
    const int N = g.N, q0 = 2 * p;
    if (q0 >= g.Q || j > N - 2 || k > N - 2) return;
    const int par = (colour + j + k) & 1;
    const int i0 = 2 * q0 + par;
    const bool v0 = i0 >= 1 && i0 <= N - 2;
    const bool v1 = q0 + 1 < g.Q && i0 + 2 <= N - 2;
    const size_t row = rowid(g, j, k), ob = (size_t)(1 - colour) * g.cs;
    const size_t me = (size_t)colour * g.cs + row + q0, xb = ob + row + q0;
    const size_t yp = ob + rowid(g, j + 1, k) + q0, ym = ob + rowid(g, j - 1, k) + q0;
    const size_t zp = ob + rowid(g, j, k + 1) + q0, zm = ob + rowid(g, j, k - 1) + q0;
    const RowIdx code = pair_codes();
    const bool zs = (mask >> 5) & 1, nz = zs && colour == 0;
    auto around = [&](const TM *d, TA (&n0)[6], TA (&n1)[6]) {
        pair_around<TM, TA>(d, par, xb, yp, ym, zp, zm, n0, n1);
#pragma unroll
        for (int x = 0; x < 6; ++x) {
            n0[x] = nz ? (TA)0 : n0[x];
            n1[x] = nz ? (TA)0 : n1[x];
        }
    };
    if (mask & 1) {
        const auto sv = ld_pair(a.ms, me), axv = ld_pair(a.ma[0], me), ayv = ld_pair(a.ma[1], me),
                   azv = ld_pair(a.ma[2], me);
        const TA s0 = (TA)sv.x, s1 = (TA)sv.y, ax0 = (TA)axv.x, ax1 = (TA)axv.y, ay0 = (TA)ayv.x, ay1 = (TA)ayv.y,
                 az0 = (TA)azv.x, az1 = (TA)azv.y;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            if ((mask >> (2 + f)) & 1) continue;
            TM *d = a.md[f];
            TA n0[6], n1[6];
            around(d, n0, n1);
            const TA sum0 = mom_off<TA>(s0, ax0, ay0, az0, code, [&](size_t x) { return n0[x]; });
            const TA sum1 = mom_off<TA>(s1, ax1, ay1, az1, code, [&](size_t x) { return n1[x]; });
            const auto oldv = ld_pair(d, me), bv = ld_pair(a.mb[f], me);
            const TA old0 = zs ? (TA)0 : (TA)oldv.x, old1 = zs ? (TA)0 : (TA)oldv.y;
            const TA dlt0 = (TA)bv.x - sum0 - old0, dlt1 = (TA)bv.y - sum1 - old1;
            st_pair(d, me, v0 ? (TM)(old0 + omega_m * dlt0) : oldv.x, v1 ? (TM)(old1 + omega_m * dlt1) : oldv.y);
            r2[f] = (v0 ? (double)dlt0 * (double)dlt0 : 0.0) + (v1 ? (double)dlt1 * (double)dlt1 : 0.0);
        }
    }
    if (mask & 2) {
        const auto axv = ld_pair(a.ta[0], me), ayv = ld_pair(a.ta[1], me), azv = ld_pair(a.ta[2], me);
        TM *d = a.td;
        TA n0[6], n1[6];
        around(d, n0, n1);
        TA den0, den1;
        const TA sum0 = theta_off<TA>(st, (TA)axv.x, (TA)ayv.x, (TA)azv.x, j, k, N, code,
                                      [&](size_t x) { return n0[x]; }, den0);
        const TA sum1 = theta_off<TA>(st, (TA)axv.y, (TA)ayv.y, (TA)azv.y, j, k, N, code,
                                      [&](size_t x) { return n1[x]; }, den1);
        const auto oldv = ld_pair(d, me), bv = ld_pair(a.tb, me);
        const TA old0 = zs ? (TA)0 : (TA)oldv.x, old1 = zs ? (TA)0 : (TA)oldv.y;
        const TA gs0 = ((TA)bv.x - sum0) / den0, gs1 = ((TA)bv.y - sum1) / den1;
        const TA dlt0 = gs0 - old0, dlt1 = gs1 - old1;
        st_pair(d, me, v0 ? (TM)(old0 + omega_t * dlt0) : oldv.x, v1 ? (TM)(old1 + omega_t * dlt1) : oldv.y);
        const double rr0 = (double)den0 * (double)dlt0, rr1 = (double)den1 * (double)dlt1;
        r2[3] = (v0 ? rr0 * rr0 : 0.0) + (v1 ? rr1 * rr1 : 0.0);
    }
}

// One launch = one colour: every thread updates two entries of a colour row.
template <typename TM, typename TA>
__global__ void __launch_bounds__(256) k_sweep(Geo g, int colour, int mask, TA omega_m, TA omega_t, TA st,
                                               SweepArgs<TM> a, double *__restrict__ partial, unsigned store,
                                               double *__restrict__ partial0, unsigned store0)
{
    const Tile tl = xcd_tile();
    const int p = tl.x * blockDim.x + threadIdx.x;
    const int j = 1 + tl.y * blockDim.y + threadIdx.y, k = 1 + tl.z;
    double r2[4] = {0.0, 0.0, 0.0, 0.0};
    sweep_pair<TM, TA>(g, colour, mask, omega_m, omega_t, st, a, p, j, k, r2);
    if (store | store0) {
        const int blk = tl.id;
        block_sum_store2<4>(r2, partial + (size_t)blk * 4, store, partial0 + (size_t)blk * 4, store0);
    }
}

// ---------------------------------------------------------------------------
// Fused multi-cavity launches.  The cavities of a batch are cut into the same
// tiles their single-cavity launches use (tx x ty threads over colour-row entries
// and rows, one tile per interior plane), numbered cavity after cavity.  A launch
// of G persistent 256-thread workgroups walks the global tile list; workgroup b
// takes tiles slot(b) + i*G with slot(b) = (b mod 8)(G/8) + b/8, so the tiles one
// XCD works on at a time are contiguous (neighbouring rows and planes share its
// L2).  A tile computes exactly what the block of the single-cavity launch with
// the same index computes, and stores its partial sums in the same record, so a
// cavity's results do not depend on the batch it is in.
// ---------------------------------------------------------------------------
struct TileMap {
    int tile0;      // first global tile of the cavity
    int tiles;      // tiles of the cavity (tiles_x * tiles_y * M)
    int tiles_x, tiles_y;
    int tx, ty;     // tile shape in threads (tx * ty = 256)
    int pad[2];
};

__device__ __forceinline__ int find_cavity(const TileMap *__restrict__ map, int ncav, int t)
{
    int lo = 0, hi = ncav - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (map[mid].tile0 <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}


template <typename TM, typename TA>
struct FusedSweepCav {
    Geo g;
    SweepArgs<TM> a;
    TA omega_m, omega_t, st;
    int plan_m, plan_t;             // sweeps of this batch per group (0: group idle)
    int skip;                       // momentum fields left alone (bits 0..2)
    int zs;                         // 1: sweep 0 of this batch starts the solve from zero
    double *part[2], *part0[2];     // partial records per colour: last sweep, first sweep
};

// One half-sweep (colour) of sweep q of the current batch, over every cavity.
template <typename TM, typename TA>
__global__ void __launch_bounds__(256) k_sweep_fused(const TileMap *__restrict__ map,
                                                     const FusedSweepCav<TM, TA> *__restrict__ cav, int ncav,
                                                     int total, int colour, int qs)
{
    const int G = gridDim.x;
    for (int t = persistent_slot(blockIdx.x, G); t < total; t += G) {
        const int c = find_cavity(map, ncav, t);
        const TileMap m = map[c];
        const FusedSweepCav<TM, TA> &cv = cav[c];
        const int mask = (qs < cv.plan_m ? 1 | (cv.skip << 2) : 0) | (qs < cv.plan_t ? 2 : 0)
                         | (qs == 0 && cv.zs ? 32 : 0);
        if (!(mask & 3)) continue;    // uniform over the workgroup
        const unsigned store = (qs == cv.plan_m - 1 ? 0x7u : 0u) | (qs == cv.plan_t - 1 ? 0x8u : 0u);
        const unsigned store0 = (qs == 0 && cv.plan_m > 1 ? 0x7u : 0u) | (qs == 0 && cv.plan_t > 1 ? 0x8u : 0u);
        const int lt = t - m.tile0;
        const int bx = lt % m.tiles_x, rest = lt / m.tiles_x;
        const int by = rest % m.tiles_y, bz = rest / m.tiles_y;
        const int tx = threadIdx.x % m.tx, ty = threadIdx.x / m.tx;
        const int p = bx * m.tx + tx, j = 1 + by * m.ty + ty, k = 1 + bz;
        double r2[4] = {0.0, 0.0, 0.0, 0.0};
        sweep_pair<TM, TA>(cv.g, colour, mask, cv.omega_m, cv.omega_t, cv.st, cv.a, p, j, k, r2);
        if (store | store0)
            block_sum_store2<4>(r2, cv.part[colour] + (size_t)lt * 4, store, cv.part0[colour] + (size_t)lt * 4,
                                store0);
        __syncthreads();    // the shared reduction buffer is reused by the next tile
    }
}

// ---------------------------------------------------------------------------
// BiCGSTAB (van der Vorst 1992) on the scaled rows, for up to four systems at once
// (u, v, w share the momentum matrix; theta has its own).  Vectors live in the
// colour layout; one launch covers both colours (blockIdx.z = 2 (k-1) + colour).
// Scalars stay on the device: sc[8*sys + {0 rho, 1 alpha, 2 omega, 3 beta,
// 4 ||r||^2, 5 breakdown flag}].  Iteration (p and v double-buffered):
//   p' = r + beta (p - omega v),  v' = B p'              alpha = rho / (rh, v')
//   s = r - alpha v',  t = B s                           omega = (t, s) / (t, t)
//   x += alpha p' + omega s,  r = s - omega t            beta = (rho'/rho)(alpha/omega)
// ---------------------------------------------------------------------------
template <typename TR, typename TM>
struct BicgArgs {
    const TR *ms, *ma[3];           // momentum rows (FP64, or FP32 in the precision mode)
    const TM *mb[3];                // momentum right-hand sides
    const TR *ta[3];                // energy rows
    const TM *tb;                   // energy right-hand side
    TM *x[4], *r[4], *rh[4], *p[4], *pn[4], *v[4], *vn[4], *t[4];
};

__device__ __forceinline__ bool bicg_node(const Geo &g, const Tile &tl, int q, int &j, int &k, int &colour,
                                          RowIdx &r)
{
    j = 1 + tl.y * blockDim.y + threadIdx.y;
    k = 1 + (tl.z >> 1);
    colour = tl.z & 1;
    return row_index(g, colour, q, j, k, r);
}

// phase 0: r = b - B x, rh = r, p = v = 0;  partials (r, r) twice
// phase 1: p' = r + beta (p - omega v), v' = B p';  partials (rh, v')
// phase 2: s = r - alpha v', t = B s;  partials (t, s), (t, t)
// phase 3: x += alpha p' + omega s, r = s - omega t;  partials (rh, r), (r, r)
template <typename TR, typename TM, typename TA>
__global__ void __launch_bounds__(256) k_bicg(Geo g, int phase, int mask, TA st, BicgArgs<TR, TM> a,
                                              const double *__restrict__ sc, double *__restrict__ partial)
{
    const Tile tl = xcd_tile();
    const int q = tl.x * blockDim.x + threadIdx.x;
    int j, k, colour;
    RowIdx r;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (bicg_node(g, tl, q, j, k, colour, r)) {
        TA ms = 0, max = 0, may = 0, maz = 0, tax = 0, tay = 0, taz = 0;
        if (mask & 1) {
            ms = (TA)a.ms[r.me]; max = (TA)a.ma[0][r.me]; may = (TA)a.ma[1][r.me]; maz = (TA)a.ma[2][r.me];
        }
        if (mask & 2) {
            tax = (TA)a.ta[0][r.me]; tay = (TA)a.ta[1][r.me]; taz = (TA)a.ta[2][r.me];
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            if (!((f < 3) ? (mask & 1) : (mask & 2))) continue;
            const double *S = sc + 8 * f;
            const TA alpha = (TA)S[1], omega = (TA)S[2], beta = (TA)S[3];
            // y -> (B y)_me for the vector given by the functor
            auto apply = [&](auto fy) -> TA {
                if (f < 3) return fy(r.me) + mom_off<TA>(ms, max, may, maz, r, fy);
                TA den;
                const TA off = theta_off<TA>(st, tax, tay, taz, j, k, g.N, r, fy, den);
                return den * fy(r.me) + off;
            };
            if (phase == 0) {
                const TM *x = a.x[f];
                const TA bx = apply([&](size_t i) { return (TA)x[i]; });
                const TA b = f < 3 ? (TA)a.mb[f][r.me] : (TA)a.tb[r.me];
                const TA rr = b - bx;
                a.r[f][r.me] = (TM)rr;
                a.rh[f][r.me] = (TM)rr;
                a.p[f][r.me] = (TM)0;
                a.v[f][r.me] = (TM)0;
                acc[2 * f] = (double)rr * (double)rr;
                acc[2 * f + 1] = acc[2 * f];
            } else if (phase == 1) {
                const TM *R = a.r[f], *P = a.p[f], *V = a.v[f];
                auto pnew = [&](size_t i) { return (TA)R[i] + beta * ((TA)P[i] - omega * (TA)V[i]); };
                const TA vv = apply(pnew);
                a.pn[f][r.me] = (TM)pnew(r.me);
                a.vn[f][r.me] = (TM)vv;
                acc[2 * f] = (double)a.rh[f][r.me] * (double)vv;
            } else if (phase == 2) {
                const TM *R = a.r[f], *V = a.vn[f];
                auto sv = [&](size_t i) { return (TA)R[i] - alpha * (TA)V[i]; };
                const TA tt = apply(sv);
                a.t[f][r.me] = (TM)tt;
                const TA s0 = sv(r.me);
                acc[2 * f] = (double)tt * (double)s0;
                acc[2 * f + 1] = (double)tt * (double)tt;
            } else {
                const size_t m = r.me;
                const TA s0 = (TA)a.r[f][m] - alpha * (TA)a.vn[f][m];
                const TA xn = (TA)a.x[f][m] + alpha * (TA)a.pn[f][m] + omega * s0;
                const TA rn = s0 - omega * (TA)a.t[f][m];
                a.x[f][m] = (TM)xn;
                a.r[f][m] = (TM)rn;
                acc[2 * f] = (double)a.rh[f][m] * (double)rn;
                acc[2 * f + 1] = (double)rn * (double)rn;
            }
        }
    }
    const int blk = tl.id;
    block_sum_store<8>(acc, partial + (size_t)blk * 8);
}

// Reduce the partial records (8 values each) of one BiCGSTAB phase in fixed order
// and update the scalars of the active systems (one block of 256 threads).
__global__ void __launch_bounds__(1024) k_bicg_scalars(int phase, int mask, const double *__restrict__ part, int nb,
                                                       double *__restrict__ sc)
{
    __shared__ double sh[8][16];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    double acc[8];
    fold_records<8>(part, nb, 0, acc);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        double s = acc[c];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) sh[c][wave] = s;
    }
    __syncthreads();
    if (t != 0) return;
    double tot[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        tot[c] = sh[c][0];
        for (int w = 1; w < 16; ++w) tot[c] += sh[c][w];
    }
    for (int f = 0; f < 4; ++f) {
        if (!((f < 3) ? (mask & 1) : (mask & 2))) continue;
        double *S = sc + 8 * f;
        const double a = tot[2 * f], b = tot[2 * f + 1];
        if (phase == 0) {
            S[0] = a; S[1] = 0.0; S[2] = 1.0; S[3] = 0.0; S[4] = b; S[5] = 0.0;
        } else if (phase == 1) {
            if (a != 0.0 && isfinite(a) && isfinite(S[0])) S[1] = S[0] / a;
            else { S[1] = 0.0; S[5] = 1.0; }
        } else if (phase == 2) {
            S[2] = (b > 0.0 && isfinite(a) && isfinite(b)) ? a / b : 0.0;
        } else {
            const double rho = a;
            if (S[0] != 0.0 && S[2] != 0.0 && isfinite(rho)) S[3] = (rho / S[0]) * (S[1] / S[2]);
            else { S[3] = 0.0; if (b > 0.0) S[5] = 1.0; }
            S[0] = rho;
            S[4] = b;
        }
    }
}

// ---------------------------------------------------------------------------
// Iterative refinement of the precision mode, one launch per outer pass over both
// colours.  The current iterate is d + e (FP64 increment plus the FP32 correction
// of the last inner solve) for the systems in `emask` (bit f: system f's
// correction is valid) and d alone for the others.  Every node forms the FP64
// residual r = b - B (d + e) of the scaled FP64 rows (so the refinement converges
// to the FP64 solution, not to that of the FP32 rows) and stores it in FP32 for
// the next inner solve, which starts from e = 0 without reading e.  A system in
// emask also has its folded iterate d + e written to the second increment buffer
// dn: folded in place, a neighbour could read a node's d + e after its fold.
// Two colour-row entries per thread as in the sweeps; per-block partial sums of
// ||r||^2 per colour.
// ---------------------------------------------------------------------------
template <typename TR>
struct RefineArgs {
    const TR *ms, *ma[3], *ta[3];   // rows (FP64)
    const double *b[4];             // right-hand sides (u, v, w, theta)
    const double *d[4];             // increments (FP64)
    double *dn[4];                  // folded increments (systems in emask)
    const float *e[4];              // corrections from the inner solve
    float *r[4];                    // residuals for the inner solve
};

template <typename TR>
__device__ __forceinline__ void refine_pair(const Geo &g, int colour, int mask, int emask, double st,
                                            const RefineArgs<TR> &a, int p, int j, int k, double (&acc)[4])
{
    const int N = g.N, q0 = 2 * p;
    if (q0 >= g.Q || j > N - 2 || k > N - 2) return;
    const int par = (colour + j + k) & 1;
    const int i0 = 2 * q0 + par;
    const bool v0 = i0 >= 1 && i0 <= N - 2;
    const bool v1 = q0 + 1 < g.Q && i0 + 2 <= N - 2;
    const size_t row = rowid(g, j, k), ob = (size_t)(1 - colour) * g.cs;
    const size_t me = (size_t)colour * g.cs + row + q0, xb = ob + row + q0;
    const size_t yp = ob + rowid(g, j + 1, k) + q0, ym = ob + rowid(g, j - 1, k) + q0;
    const size_t zp = ob + rowid(g, j, k + 1) + q0, zm = ob + rowid(g, j, k - 1) + q0;
    const RowIdx code = pair_codes();
    double2 sv{0.0, 0.0}, axv{0.0, 0.0}, ayv{0.0, 0.0}, azv{0.0, 0.0};
    if (mask & 1) {
        sv = ld_pair(a.ms, me);
        axv = ld_pair(a.ma[0], me);
        ayv = ld_pair(a.ma[1], me);
        azv = ld_pair(a.ma[2], me);
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        if (!((f < 3) ? (mask & 1) : (mask & 2))) continue;
        const bool fold = (emask >> f) & 1;
        double n0[6], n1[6];
        pair_around<double, double>(a.d[f], par, xb, yp, ym, zp, zm, n0, n1);
        const auto dv = ld_pair(a.d[f], me);
        double own0 = dv.x, own1 = dv.y;
        if (fold) {
            double e0[6], e1[6];
            pair_around<float, double>(a.e[f], par, xb, yp, ym, zp, zm, e0, e1);
#pragma unroll
            for (int x = 0; x < 6; ++x) {
                n0[x] += e0[x];
                n1[x] += e1[x];
            }
            const auto ev = ld_pair(a.e[f], me);
            own0 += (double)ev.x;
            own1 += (double)ev.y;
        }
        double bx0, bx1;
        if (f < 3) {
            bx0 = own0 + mom_off<double>((double)sv.x, (double)axv.x, (double)ayv.x, (double)azv.x, code,
                                         [&](size_t x) { return n0[x]; });
            bx1 = own1 + mom_off<double>((double)sv.y, (double)axv.y, (double)ayv.y, (double)azv.y, code,
                                         [&](size_t x) { return n1[x]; });
        } else {
            const auto axv = ld_pair(a.ta[0], me), ayv = ld_pair(a.ta[1], me), azv = ld_pair(a.ta[2], me);
            double den0, den1;
            const double off0 = theta_off<double>(st, (double)axv.x, (double)ayv.x, (double)azv.x, j, k, N, code,
                                                  [&](size_t x) { return n0[x]; }, den0);
            const double off1 = theta_off<double>(st, (double)axv.y, (double)ayv.y, (double)azv.y, j, k, N, code,
                                                  [&](size_t x) { return n1[x]; }, den1);
            bx0 = den0 * own0 + off0;
            bx1 = den1 * own1 + off1;
        }
        const auto bv = ld_pair(a.b[f], me);
        const double rr0 = bv.x - bx0, rr1 = bv.y - bx1;
        st_pair(a.r[f], me, v0 ? (float)rr0 : 0.0f, v1 ? (float)rr1 : 0.0f);
        if (fold) st_pair(a.dn[f], me, v0 ? own0 : dv.x, v1 ? own1 : dv.y);
        acc[f] = (v0 ? rr0 * rr0 : 0.0) + (v1 ? rr1 * rr1 : 0.0);
    }
}

// Tiles of the sweep launch's shape for both colours: tile z = 2 (k - 1) + colour,
// so the run of tiles an XCD takes holds both colours of its planes.  The record
// of a tile is its index within its colour.
template <typename TR>
__global__ void __launch_bounds__(256) k_refine_pass(Geo g, int mask, int emask, double st, RefineArgs<TR> a,
                                                     double *__restrict__ part_r, double *__restrict__ part_b)
{
    const Tile tl = xcd_tile();
    const int colour = tl.z & 1, kz = tl.z >> 1;
    const int p = tl.x * blockDim.x + threadIdx.x;
    const int j = 1 + tl.y * blockDim.y + threadIdx.y, k = 1 + kz;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    refine_pair<TR>(g, colour, mask, emask, st, a, p, j, k, acc);
    const int blk = tl.x + (int)gridDim.x * (tl.y + (int)gridDim.y * kz);
    block_sum_store<4>(acc, (colour ? part_b : part_r) + (size_t)blk * 4);
}

template <typename TR>
struct FusedRefineCav {
    Geo g;
    RefineArgs<TR> a;
    double st;
    int mask;                       // groups refined (0: cavity idle)
    int emask;                      // systems whose correction is folded
    double *part[2];                // partial records per colour
};

// One outer pass over every cavity: global tile t is colour t & 1 of the sweep
// tile t >> 1 of the batch's tile list.
template <typename TR>
__global__ void __launch_bounds__(256) k_refine_fused(const TileMap *__restrict__ map,
                                                      const FusedRefineCav<TR> *__restrict__ cav, int ncav, int total)
{
    const int G = gridDim.x;
    for (int t = persistent_slot(blockIdx.x, G); t < 2 * total; t += G) {
        const int base = t >> 1, colour = t & 1;
        const int c = find_cavity(map, ncav, base);
        const TileMap m = map[c];
        const FusedRefineCav<TR> &cv = cav[c];
        if (!cv.mask) continue;
        const int lt = base - m.tile0;
        const int bx = lt % m.tiles_x, rest = lt / m.tiles_x;
        const int by = rest % m.tiles_y, bz = rest / m.tiles_y;
        const int tx = threadIdx.x % m.tx, ty = threadIdx.x / m.tx;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        refine_pair<TR>(cv.g, colour, cv.mask, cv.emask, cv.st, cv.a, bx * m.tx + tx, 1 + by * m.ty + ty, 1 + bz,
                        acc);
        block_sum_store<4>(acc, cv.part[colour] + (size_t)lt * 4);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Update chi^{n+1} = chi^n + dchi at interior nodes.  u, v, w go to new buffers
// (the old level becomes level n-1); theta is updated in place.  Partial sums:
// ||du||^2, ||dv||^2, ||dw||^2, ||dtheta||^2, ||u'||^2, ||v'||^2, ||w'||^2, ||theta'||^2.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_update(Geo g, const double *__restrict__ u, const double *__restrict__ v,
                                                const double *__restrict__ w, double *__restrict__ un,
                                                double *__restrict__ vn, double *__restrict__ wn,
                                                double *__restrict__ T, const double *__restrict__ du,
                                                const double *__restrict__ dv, const double *__restrict__ dw,
                                                const double *__restrict__ dT, double *__restrict__ partial)
{
    const Tile tl = xcd_tile();
    const int i = 1 + tl.x * blockDim.x + threadIdx.x, j = 1 + tl.y * blockDim.y + threadIdx.y, k = 1 + tl.z;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (i <= g.N - 2 && j <= g.N - 2) {
        const size_t c = nid(g, i, j, k);
        const size_t idx = (size_t)((i + j + k) & 1) * g.cs + rowid(g, j, k) + (i >> 1);
        const double a = du[idx], b = dv[idx], e = dw[idx], t = dT[idx];
        const double nu = u[c] + a, nv = v[c] + b, nw = w[c] + e, nt = T[c] + t;
        un[c] = nu;
        vn[c] = nv;
        wn[c] = nw;
        T[c] = nt;
        acc[0] = a * a; acc[1] = b * b; acc[2] = e * e; acc[3] = t * t;
        acc[4] = nu * nu; acc[5] = nv * nv; acc[6] = nw * nw; acc[7] = nt * nt;
    }
    const int blk = tl.id;
    block_sum_store<8>(acc, partial + (size_t)blk * 8);
}

// ---------------------------------------------------------------------------
// Wall closures.  Every wall node is owned by the first face (x0, x1, y0, y1, z0,
// z1) that contains it; thread (a, b, f) handles the node (a, b) of face f.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool face_node(int N, int a, int b, int f, int &i, int &j, int &k)
{
    const int e = (f & 1) ? N - 1 : 0;
    if (f < 2) { i = e; j = a; k = b; return true; }
    if (f < 4) { i = a; j = e; k = b; return !(a == 0 || a == N - 1); }
    i = a; j = b; k = e;
    return !(a == 0 || a == N - 1 || b == 0 || b == N - 1);
}

// theta on the y/z walls at interior x: z walls at interior y first, then y walls
// at every z, each by f_0 = (4 f_1 - f_2)/3 (composed here from interior values).
__device__ __forceinline__ double theta_z_closed(const Geo &g, const double *T, int i, int j, int k)
{
    const int N = g.N;
    if (k == 0) return (4.0 * T[nid(g, i, j, 1)] - T[nid(g, i, j, 2)]) / 3.0;
    if (k == N - 1) return (4.0 * T[nid(g, i, j, N - 2)] - T[nid(g, i, j, N - 3)]) / 3.0;
    return T[nid(g, i, j, k)];
}
__device__ __forceinline__ double theta_closed(const Geo &g, const double *T, int i, int j, int k)
{
    const int N = g.N;
    if (j == 0) return (4.0 * theta_z_closed(g, T, i, 1, k) - theta_z_closed(g, T, i, 2, k)) / 3.0;
    if (j == N - 1) return (4.0 * theta_z_closed(g, T, i, N - 2, k) - theta_z_closed(g, T, i, N - 3, k)) / 3.0;
    return theta_z_closed(g, T, i, j, k);
}

// Impose the theta walls; partial sums of (new - old)^2 and new^2 over wall nodes.
// One 64 x 4 block of the face launch: its node (a, b) on face f, its record blk.
__device__ __forceinline__ void theta_walls_block(const Geo &g, const Phys &P, double *__restrict__ T,
                                                  double *__restrict__ partial, int a, int b, int f, int blk)
{
    double acc[2] = {0.0, 0.0};
    int i, j, k;
    if (a < g.N && b < g.N && face_node(g.N, a, b, f, i, j, k)) {
        const size_t c = nid(g, i, j, k);
        double nv;
        if (i == 0) nv = P.theta_hot;
        else if (i == g.N - 1) nv = P.theta_cold;
        else nv = theta_closed(g, T, i, j, k);
        const double d = nv - T[c];
        T[c] = nv;
        acc[0] = d * d;
        acc[1] = nv * nv;
    }
    block_sum_store<2>(acc, partial + (size_t)blk * 2);
}
__global__ void __launch_bounds__(256) k_theta_walls(Geo g, Phys P, double *__restrict__ T, double *__restrict__ partial)
{
    theta_walls_block(g, P, T, partial, blockIdx.x * blockDim.x + threadIdx.x, blockIdx.y * blockDim.y + threadIdx.y,
                      blockIdx.z, blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z));
}

// p walls: x faces at interior (j,k), then y faces at every x and interior z, then z
// faces everywhere, each by f_0 = (4 f_1 - f_2)/3 (composed from interior values).
__device__ __forceinline__ double p_x_closed(const Geo &g, const double *p, int i, int j, int k)
{
    const int N = g.N;
    if (i == 0) return (4.0 * p[nid(g, 1, j, k)] - p[nid(g, 2, j, k)]) / 3.0;
    if (i == N - 1) return (4.0 * p[nid(g, N - 2, j, k)] - p[nid(g, N - 3, j, k)]) / 3.0;
    return p[nid(g, i, j, k)];
}
__device__ __forceinline__ double p_y_closed(const Geo &g, const double *p, int i, int j, int k)
{
    const int N = g.N;
    if (j == 0) return (4.0 * p_x_closed(g, p, i, 1, k) - p_x_closed(g, p, i, 2, k)) / 3.0;
    if (j == N - 1) return (4.0 * p_x_closed(g, p, i, N - 2, k) - p_x_closed(g, p, i, N - 3, k)) / 3.0;
    return p_x_closed(g, p, i, j, k);
}
__device__ __forceinline__ double p_closed(const Geo &g, const double *p, int i, int j, int k)
{
    const int N = g.N;
    if (k == 0) return (4.0 * p_y_closed(g, p, i, j, 1) - p_y_closed(g, p, i, j, 2)) / 3.0;
    if (k == N - 1) return (4.0 * p_y_closed(g, p, i, j, N - 2) - p_y_closed(g, p, i, j, N - 3)) / 3.0;
    return p_y_closed(g, p, i, j, k);
}

__device__ __forceinline__ void p_walls_node(const Geo &g, double *__restrict__ p, int a, int b, int f)
{
    int i, j, k;
    if (a < g.N && b < g.N && face_node(g.N, a, b, f, i, j, k)) p[nid(g, i, j, k)] = p_closed(g, p, i, j, k);
}
__global__ void __launch_bounds__(256) k_p_walls(Geo g, double *__restrict__ p)
{
    p_walls_node(g, p, blockIdx.x * blockDim.x + threadIdx.x, blockIdx.y * blockDim.y + threadIdx.y, blockIdx.z);
}

// No-slip walls (velocity 0) for set_state with boundary conditions.
__global__ void __launch_bounds__(256) k_zero_walls(Geo g, double *__restrict__ u, double *__restrict__ v,
                                                    double *__restrict__ w)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x, b = blockIdx.y * blockDim.y + threadIdx.y, f = blockIdx.z;
    int i, j, k;
    if (a < g.N && b < g.N && face_node(g.N, a, b, f, i, j, k)) {
        const size_t c = nid(g, i, j, k);
        u[c] = 0.0; v[c] = 0.0; w[c] = 0.0;
    }
}

// ---------------------------------------------------------------------------
// Modified artificial compressibility (Sec. 2.2): D = div v^{n+1} by central
// differences at interior nodes, p <- p - lambda D (when apply != 0); partial max |D|.
// ---------------------------------------------------------------------------
// One 64 x 4 tile of the interior launch (thread (tx, ty) of it).
__device__ __forceinline__ void divergence_tile(const Geo &g, const Phys &P, const Tile &tl, int tx, int ty,
                                                const double *__restrict__ u, const double *__restrict__ v,
                                                const double *__restrict__ w, double *__restrict__ p,
                                                double *__restrict__ dstore, int apply, double *__restrict__ partial)
{
    const int i = 1 + tl.x * 64 + tx, j = 1 + tl.y * 4 + ty, k = 1 + tl.z;
    double acc[1] = {0.0};
    if (i <= g.N - 2 && j <= g.N - 2) {
        const size_t c = nid(g, i, j, k), sy = (size_t)g.N, sz = (size_t)g.N * g.N;
        const double D = (u[c + 1] - u[c - 1]) * g.inv2h + (v[c + sy] - v[c - sy]) * g.inv2h
                         + (w[c + sz] - w[c - sz]) * g.inv2h;
        acc[0] = fabs(D);
        if (apply) p[c] -= P.lambda * D;
        if (dstore) dstore[c] = D;
    }
    const int blk = tl.id;
    block_max_store<1>(acc, partial + blk);
}

// Divergence of a trial velocity level n + increment (the increments in the
// colour-split layout, zero on the walls), for the pressure iterations of a step:
// the same sums as k_update followed by k_divergence, so the value is identical to
// the one the step measures once the trial is accepted.  D into dstore, partial
// max |D|.
__device__ __forceinline__ double trial_vel(const Geo &g, const double *__restrict__ f,
                                            const double *__restrict__ df, int i, int j, int k)
{
    const double x = f[nid(g, i, j, k)];
    if (i < 1 || i > g.N - 2 || j < 1 || j > g.N - 2 || k < 1 || k > g.N - 2) return x;
    return x + df[(size_t)((i + j + k) & 1) * g.cs + rowid(g, j, k) + (i >> 1)];
}

__global__ void __launch_bounds__(256) k_divergence_trial(Geo g, const double *__restrict__ u,
                                                          const double *__restrict__ v, const double *__restrict__ w,
                                                          const double *__restrict__ du, const double *__restrict__ dv,
                                                          const double *__restrict__ dw, double *__restrict__ dstore,
                                                          double *__restrict__ partial)
{
    const Tile tl = xcd_tile();
    const int i = 1 + tl.x * blockDim.x + threadIdx.x, j = 1 + tl.y * blockDim.y + threadIdx.y, k = 1 + tl.z;
    double acc[1] = {0.0};
    if (i <= g.N - 2 && j <= g.N - 2) {
        const double D = (trial_vel(g, u, du, i + 1, j, k) - trial_vel(g, u, du, i - 1, j, k)) * g.inv2h
                         + (trial_vel(g, v, dv, i, j + 1, k) - trial_vel(g, v, dv, i, j - 1, k)) * g.inv2h
                         + (trial_vel(g, w, dw, i, j, k + 1) - trial_vel(g, w, dw, i, j, k - 1)) * g.inv2h;
        acc[0] = fabs(D);
        dstore[nid(g, i, j, k)] = D;
    }
    const int blk = tl.id;
    block_max_store<1>(acc, partial + blk);
}

// p <- p - lambda D from a stored divergence (when the correction is gated by a
// positive tolerance the decision needs the global max first).
__global__ void __launch_bounds__(256) k_pressure_apply(Geo g, Phys P, const double *__restrict__ dstore,
                                                        double *__restrict__ p)
{
    const Tile tl = xcd_tile();
    const int i = 1 + tl.x * blockDim.x + threadIdx.x, j = 1 + tl.y * blockDim.y + threadIdx.y, k = 1 + tl.z;
    if (i <= g.N - 2 && j <= g.N - 2) {
        const size_t c = nid(g, i, j, k);
        p[c] -= P.lambda * dstore[c];
    }
}

// ---------------------------------------------------------------------------
// Probes (the monitoring points of the grid-independence study, Sec. 3.1): u, v,
// w, theta, p of level n at points of the closed unit cube by trilinear
// interpolation of the eight surrounding nodes.  xyz[3q..3q+2] in [0, 1] (checked
// by the caller), out[5q..5q+4].
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_probe(Geo g, const double *__restrict__ u, const double *__restrict__ v,
                                               const double *__restrict__ w, const double *__restrict__ T,
                                               const double *__restrict__ p, const double *__restrict__ xyz, int n,
                                               double *__restrict__ out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    int c0[3];
    double t[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double f = xyz[3 * q + d] * (double)(g.N - 1);
        const int i = min(max((int)floor(f), 0), g.N - 2);     // the last cell holds the far wall
        c0[d] = i;
        t[d] = f - (double)i;
    }
    const double *fld[5] = {u, v, w, T, p};
    double acc[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int corner = 0; corner < 8; ++corner) {
        const int a = corner & 1, b = (corner >> 1) & 1, c = corner >> 2;
        const double wgt = (a ? t[0] : 1.0 - t[0]) * (b ? t[1] : 1.0 - t[1]) * (c ? t[2] : 1.0 - t[2]);
        const size_t id = nid(g, c0[0] + a, c0[1] + b, c0[2] + c);
#pragma unroll
        for (int f = 0; f < 5; ++f) acc[f] += wgt * fld[f][id];
    }
#pragma unroll
    for (int f = 0; f < 5; ++f) out[5 * q + f] = acc[f];
}

// Nusselt numbers of one z-row k of both x-walls (Sec. 4.2): Nu_local = -dtheta/dx by
// the 5-point one-sided 4th-order formula at every y-node j (stored at j + N k),
// Nu_avg(z_k) = the Simpson-weighted sum over y, and the row's largest hot-wall
// Nu_local.  One block of 256 threads per row; thread t takes j = t, t + 256, ... in
// order, then fixed-order trees over the block: deterministic.
__device__ __forceinline__ void nu_row_block(const Geo &g, const double *__restrict__ wq, const double *__restrict__ T,
                                             double *__restrict__ nuh, double *__restrict__ nuc,
                                             double *__restrict__ avh, double *__restrict__ avc,
                                             double *__restrict__ mxh, int k)
{
    __shared__ double sh[3][256];
    const int t = threadIdx.x, N = g.N;
    const double inv12h = 1.0 / (12.0 * g.h);
    double a = 0.0, c = 0.0, m = -HUGE_VAL;
    for (int j = t; j < N; j += 256) {
        const double dh = (-25.0 * T[nid(g, 0, j, k)] + 48.0 * T[nid(g, 1, j, k)] - 36.0 * T[nid(g, 2, j, k)]
                           + 16.0 * T[nid(g, 3, j, k)] - 3.0 * T[nid(g, 4, j, k)]) * inv12h;
        const double dc = (25.0 * T[nid(g, N - 1, j, k)] - 48.0 * T[nid(g, N - 2, j, k)]
                           + 36.0 * T[nid(g, N - 3, j, k)] - 16.0 * T[nid(g, N - 4, j, k)]
                           + 3.0 * T[nid(g, N - 5, j, k)]) * inv12h;
        const double nh = -dh, nc = -dc;
        nuh[j + (size_t)N * k] = nh;
        nuc[j + (size_t)N * k] = nc;
        a += wq[j] * nh;
        c += wq[j] * nc;
        m = nanmax(m, nh);
    }
    sh[0][t] = a;
    sh[1][t] = c;
    sh[2][t] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            sh[0][t] += sh[0][t + w];
            sh[1][t] += sh[1][t + w];
            sh[2][t] = nanmax(sh[2][t], sh[2][t + w]);
        }
        __syncthreads();
    }
    if (t == 0) {
        avh[k] = sh[0][0];
        avc[k] = sh[1][0];
        mxh[k] = sh[2][0];
    }
}
__global__ void __launch_bounds__(256) k_nu_rows(Geo g, const double *__restrict__ wq, const double *__restrict__ T,
                                                 double *__restrict__ nuh, double *__restrict__ nuc,
                                                 double *__restrict__ avh, double *__restrict__ avc,
                                                 double *__restrict__ mxh)
{
    nu_row_block(g, wq, T, nuh, nuc, avh, avc, mxh, blockIdx.x);
}

// Means over z (Simpson), maxima over z of Nu_avg, and the max of the local
// hot-wall Nu (over the rows' maxima): one block of 1024 threads, fixed-order trees.
__device__ __forceinline__ void nu_final_block(const Geo &g, const double *__restrict__ wq,
                                               const double *__restrict__ avh, const double *__restrict__ avc,
                                               const double *__restrict__ mxh, double *__restrict__ out,
                                               double *__restrict__ out_host = nullptr)
{
    __shared__ double sh[5][16];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    double v[5] = {0.0, 0.0, -HUGE_VAL, -HUGE_VAL, -HUGE_VAL};
    for (int k = t; k < g.N; k += 1024) {
        v[0] += wq[k] * avh[k];
        v[1] += wq[k] * avc[k];
        v[2] = nanmax(v[2], avh[k]);
        v[3] = nanmax(v[3], avc[k]);
        v[4] = nanmax(v[4], mxh[k]);
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        double x = v[c];
        for (int off = 32; off > 0; off >>= 1) {
            const double y = __shfl_down(x, off, 64);
            x = c < 2 ? x + y : nanmax(x, y);
        }
        if (lane == 0) sh[c][wave] = x;
    }
    __syncthreads();
    if (t < 5) {
        double x = sh[t][0];
        for (int w = 1; w < 16; ++w) x = t < 2 ? x + sh[t][w] : nanmax(x, sh[t][w]);
        out[t] = x;
        if (out_host) store_host(out_host + t, x);
    }
}
__global__ void __launch_bounds__(1024) k_nu_final(Geo g, const double *__restrict__ wq, const double *__restrict__ avh,
                                                   const double *__restrict__ avc, const double *__restrict__ mxh,
                                                   double *__restrict__ out)
{
    nu_final_block(g, wq, avh, avc, mxh, out);
}

// Entropy generation (Sec. 4.3): E_HT = |grad theta|^2, E_FF = phi eta I2 with eta
// from the current velocity, E_local = E_HT + E_FF, Be_local = E_HT / E_local (1
// where E_local = 0).  Partial Simpson-weighted sums of E_HT, E_FF and Be_local.
// eta_out (optional) receives eta, computed exactly as k_eta computes it: run at
// the end of a step on the new velocities, it supplies the next step's viscosity
// (with eta_prev, relaxed: relax eta + (1 - relax) eta_prev).
// Composite Simpson weights on the N nodes of [0, 1] (Simpson's 3/8 rule on the
// last three intervals when N-1 is odd), one thread per node, each weight summed
// from its panels in the order the host builds them (left panel's end first), so
// the values are bitwise those of the host table.
__global__ void __launch_bounds__(256) k_simpson_weights(int N, double *__restrict__ wq)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const double h = 1.0 / (N - 1);
    const int nint = N - 1;
    const int n13 = (nint % 2 == 0) ? nint : nint - 3;
    double w = 0.0;
    if (q <= n13) {
        if (q & 1) {
            w += 4.0 * h / 3.0;
        } else {
            if (q >= 2) w += h / 3.0;        // right end of the panel [q-2, q]
            if (q + 2 <= n13) w += h / 3.0;  // left end of the panel [q, q+2]
        }
    }
    if (n13 != nint && q >= n13) {
        const int r = q - n13;
        w += (r == 0 || r == 3) ? 3.0 * h / 8.0 : 9.0 * h / 8.0;
    }
    wq[q] = w;
}

// The hosc_diag record (declaration order) from the Nusselt outputs nu[0..4] and
// the entropy sums ent[0..2], with the arithmetic of the host's record.
__global__ void k_diag_pack(const double *__restrict__ nu, const double *__restrict__ ent, double *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double e_total = ent[0] + ent[1];
    out[0] = nu[0];
    out[1] = nu[1];
    out[2] = nu[2];
    out[3] = nu[3];
    out[4] = e_total;
    out[5] = ent[0];
    out[6] = ent[1];
    out[7] = e_total > 0.0 ? ent[0] / e_total : 1.0;
    out[8] = ent[2];
    out[9] = nu[4];
}

// One 256-node block (tile tl) of the all-node launch.
__device__ __forceinline__ void entropy_block(const Geo &g, const Phys &P, const Tile &tl, const double *__restrict__ wq,
                                             const double *__restrict__ u, const double *__restrict__ v,
                                             const double *__restrict__ w, const double *__restrict__ T,
                                             double *__restrict__ el, double *__restrict__ bl,
                                             double *__restrict__ eta_out, double *__restrict__ partial,
                                             const double *__restrict__ eta_prev, double relax)
{
    int i, j, k;
    double acc[3] = {0.0, 0.0, 0.0};
    if (all_node(g, tl, i, j, k)) {
        const size_t c = nid(g, i, j, k), sy = (size_t)g.N, sz = (size_t)g.N * g.N;
        const double Tc = T[c];
        const double tx = dnode(T, Tc, c, 1, i, g.N, g.inv2h), ty = dnode(T, Tc, c, sy, j, g.N, g.inv2h),
                     tz = dnode(T, Tc, c, sz, k, g.N, g.inv2h);
        const double eht = tx * tx + ty * ty + tz * tz;
        const VelGrad d = vel_grad(g, u, v, w, i, j, k);
        const double I2 = strain_I2(d);
        const double eta = pow(fmax(I2, P.i2_floor), P.ex);    // as k_eta computes it
        if (eta_out) eta_out[c] = eta_prev ? relax * eta + (1.0 - relax) * eta_prev[c] : eta;
        const double eff = P.phi * eta * I2;
        const double e = eht + eff;
        const double be = e > 0.0 ? eht / e : 1.0;
        const double wv = wq[i] * wq[j] * wq[k];
        acc[0] = wv * eht;
        acc[1] = wv * eff;
        acc[2] = wv * be;
        if (el) el[c] = e;
        if (bl) bl[c] = be;
    }
    const int blk = tl.id;
    block_sum_store<3>(acc, partial + (size_t)blk * 3);
}
__global__ void __launch_bounds__(256) k_entropy(Geo g, Phys P, const double *__restrict__ wq,
                                                 const double *__restrict__ u, const double *__restrict__ v,
                                                 const double *__restrict__ w, const double *__restrict__ T,
                                                 double *__restrict__ el, double *__restrict__ bl,
                                                 double *__restrict__ eta_out, double *__restrict__ partial,
                                                 const double *__restrict__ eta_prev = nullptr, double relax = 1.0)
{
    entropy_block(g, P, xcd_tile(), wq, u, v, w, T, el, bl, eta_out, partial, eta_prev, relax);
}

// ---------------------------------------------------------------------------
// The end of a step in three launches.  The blocks of one launch take different
// roles, each block computing exactly what the same block of that role's own
// launch computes (same tile, same thread layout, same partial record), so the
// results are bitwise those of the separate launches; the roles of one launch do
// not read what another role of it writes.
// ---------------------------------------------------------------------------

// Blocks [0, nd): divergence of the new velocity and, with apply, p <- p - lambda D
// (the 64 x 4 interior tiles, grid dgx x dgy x (N-2)); blocks [nd, nd + nf): the
// theta walls (the 64 x 4 face blocks, grid fgx x fgy x 6).
__global__ void __launch_bounds__(256) k_tail_div_walls(Geo g, Phys P, const double *__restrict__ u,
                                                        const double *__restrict__ v, const double *__restrict__ w,
                                                        double *__restrict__ p, double *__restrict__ dstore, int apply,
                                                        double *__restrict__ part_div, int dgx, int dgy, int nd,
                                                        double *__restrict__ T, double *__restrict__ part_walls,
                                                        int fgx, int fgy)
{
    const int b = blockIdx.x, t = threadIdx.x;
    if (b < nd) {
        divergence_tile(g, P, xcd_tile_of(b, nd, dgx, dgy), t & 63, t >> 6, u, v, w, p, dstore, apply, part_div);
    } else {
        const int q = b - nd, bx = q % fgx, by = (q / fgx) % fgy, f = q / (fgx * fgy);
        theta_walls_block(g, P, T, part_walls, bx * 64 + (t & 63), by * 4 + (t >> 6), f, q);
    }
}

// Blocks [0, ne): the entropy pass over every node (it also writes the next step's
// viscosity); [ne, ne + nf): the pressure walls (when the correction was applied
// in the previous launch; nf = 0 otherwise); then one block per z-row of the
// Nusselt numbers.
__global__ void __launch_bounds__(256) k_tail_diag(Geo g, Phys P, const double *__restrict__ wq,
                                                   const double *__restrict__ u, const double *__restrict__ v,
                                                   const double *__restrict__ w, const double *__restrict__ T,
                                                   double *__restrict__ eta_out, double *__restrict__ part_ent,
                                                   const double *__restrict__ eta_prev, double relax, int ne,
                                                   double *__restrict__ p, int nf, int fgx, int fgy,
                                                   double *__restrict__ nuh, double *__restrict__ nuc,
                                                   double *__restrict__ avh, double *__restrict__ avc,
                                                   double *__restrict__ mxh)
{
    const int b = blockIdx.x, t = threadIdx.x;
    if (b < ne) {
        entropy_block(g, P, xcd_tile_of(b, ne, ne, 1), wq, u, v, w, T, nullptr, nullptr, eta_out, part_ent, eta_prev,
                      relax);
    } else if (b < ne + nf) {
        const int q = b - ne, bx = q % fgx, by = (q / fgx) % fgy, f = q / (fgx * fgy);
        p_walls_node(g, p, bx * 64 + (t & 63), by * 4 + (t >> 6), f);
    } else {
        nu_row_block(g, wq, T, nuh, nuc, avh, avc, mxh, b - ne - nf);
    }
}

// Blocks [0, n): the reductions of the step's partial sums; block n: the Nusselt
// means and maxima.
// nu_host (may be null): the Nusselt outputs to mapped host memory as well.
__global__ void __launch_bounds__(1024) k_tail_reduce(ReduceJobs4 jobs, int n, Geo g, const double *__restrict__ wq,
                                                      const double *__restrict__ avh, const double *__restrict__ avc,
                                                      const double *__restrict__ mxh, double *__restrict__ nu_out,
                                                      double *__restrict__ nu_host)
{
    if ((int)blockIdx.x < n) {
        const ReduceJob &jb = jobs.j[blockIdx.x];
        reduce_block(jb.part, jb.nb, jb.nc, jb.op, jb.out, jb.out_host);
    } else {
        nu_final_block(g, wq, avh, avc, mxh, nu_out, nu_host);
    }
}

// STREAM-style copy (16-byte accesses, grid-stride): measures the achievable
// HBM bandwidth and calibrates hardware traffic counters against known bytes.
__global__ void __launch_bounds__(256) k_copy(const double2 *__restrict__ src, double2 *__restrict__ dst, size_t n)
{
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x)
        dst[q] = src[q];
}

// Up to four device-to-device copies of n 16-byte elements in one grid-stride launch.
struct Copies4 {
    const double2 *src[4];
    double2 *dst[4];
    int count;
};
__global__ void __launch_bounds__(256) k_copy4(Copies4 c, size_t n)
{
    for (int a = 0; a < c.count; ++a)
        for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n; q += (size_t)gridDim.x * blockDim.x)
            c.dst[a][q] = c.src[a][q];
}

}  // namespace hosc
