// hosc.hip -- host runtime and C ABI of libhosc (declared in include/hosc.h).
//
// One solver = one cavity on one device.  All device memory comes from the
// caller's workspace; the runtime carves it into natural-layout fields (levels n
// and n-1, viscosity, momentum sources) and colour-layout rows of the implicit
// systems, and drives the step of Sec. 2.2 of the paper on the caller's stream:
//   eta, E*  ->  HOSC assembly  ->  red-black SOR sweeps (both systems together,
//   convergence measured inside the sweeps)  ->  update + walls + steady residual
//   ->  divergence and pressure correction + pressure walls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <deque>
#include <map>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hosc.h"
#include "hosc_kernels.hpp"
#include "hosc_probes.hpp"

using namespace hosc;

namespace {

constexpr size_t kAlign = 256;
constexpr int kRed = 64;    // doubles in the reduction output block

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Launch {
    dim3 blk_all, grd_all;      // every node (natural layout)
    dim3 blk_int, grd_int;      // interior nodes (natural layout)
    dim3 blk_sw, grd_sw;        // one colour of the interior (colour layout)
    dim3 blk_face, grd_face;    // wall nodes, 6 faces
    dim3 grd_bc;                // both colours of the interior (BiCGSTAB)
    dim3 blk_sp, grd_sp;        // one colour of the interior, two colour-row entries per thread (sweeps)
    size_t nb_int, nb_sw, nb_face, nb_all, nb_bc, nb_sp;
};

// Workspace map (element counts in doubles, each region 256-byte aligned).
struct Layout {
    size_t n3, cs;
    size_t natural_arrays = 17;   // u v w T p u2 v2 w2 eta etap E3 Ep3 dbg
    size_t colour_arrays = 15;    // ms ma3 mb3 md3 ta3 tb td (each 2 colours)
    size_t bicg_arrays = 0;       // r rh p pn v vn t for 4 systems (BiCGSTAB enabled)
    size_t fp32_arrays = 0;       // precision mode: FP32 rows (7), residuals and corrections of 4 systems
    size_t alt_arrays = 0;        // precision mode: second FP64 increment buffers of the refinement (4 systems)
    size_t partial;               // partial-sum records
    size_t total_bytes;
};

Geo make_geo(int N)
{
    Geo g;
    g.N = N;
    g.H = (N + 1) / 2;
    g.H += g.H & 1;     // even row length: the sweeps load entries in aligned pairs
    g.Q = ((N - 2) >> 1) + 1;
    g.pad = 0;
    g.h = 1.0 / (N - 1);
    g.h2 = g.h * g.h;
    g.inv2h = 1.0 / (2.0 * g.h);
    g.invh2 = 1.0 / g.h2;
    g.h2_12 = g.h2 / 12.0;
    g.inv3h = 1.0 / (3.0 * g.h);
    g.inv12h = 1.0 / (12.0 * g.h);
    g.inv6h2 = 1.0 / (6.0 * g.h2);
    g.invN = 1.0 / N;
    g.n3 = (size_t)N * N * N;
    g.cs = (size_t)N * N * g.H;
    return g;
}

Launch make_launch(const Geo &g)
{
    Launch L;
    const int N = g.N, M = N - 2;
    L.blk_all = dim3(256, 1, 1);
    L.grd_all = dim3((unsigned)((g.n3 + 255) / 256), 1, 1);
    L.blk_int = dim3(64, 4, 1);
    L.grd_int = dim3((M + 63) / 64, (M + 3) / 4, M);
    int bx = 64;
    while (bx > 8 && bx / 2 >= g.Q) bx /= 2;
    // rows longer than 64 entries whose last 64-wide tile would be at most half
    // used take 32-wide tiles (161^3: 3.7 -> 4.6 TB/s per half-sweep)
    if (bx == 64 && g.Q % 64 != 0 && g.Q % 64 <= 32) bx = 32;
    L.blk_sw = dim3(bx, 256 / bx, 1);
    L.grd_sw = dim3((g.Q + bx - 1) / bx, (M + L.blk_sw.y - 1) / L.blk_sw.y, M);
    L.blk_face = dim3(64, 4, 1);
    L.grd_face = dim3((N + 63) / 64, (N + 3) / 4, 6);
    L.nb_all = (size_t)L.grd_all.x * L.grd_all.y * L.grd_all.z;
    L.nb_int = (size_t)L.grd_int.x * L.grd_int.y * L.grd_int.z;
    L.nb_sw = (size_t)L.grd_sw.x * L.grd_sw.y * L.grd_sw.z;
    L.nb_face = (size_t)L.grd_face.x * L.grd_face.y * L.grd_face.z;
    L.grd_bc = dim3(L.grd_sw.x, L.grd_sw.y, 2 * M);
    L.nb_bc = (size_t)L.grd_bc.x * L.grd_bc.y * L.grd_bc.z;
    // sweeps: pairs of colour-row entries, P per row; the same narrowing of the
    // tile for short or ragged rows
    const int P = (g.Q + 1) / 2;
    int px = 64;
    while (px > 8 && px / 2 >= P) px /= 2;
    if (px == 64 && P % 64 != 0 && P % 64 <= 32) px = 32;
    L.blk_sp = dim3(px, 256 / px, 1);
    L.grd_sp = dim3((P + px - 1) / px, (M + L.blk_sp.y - 1) / L.blk_sp.y, M);
    L.nb_sp = (size_t)L.grd_sp.x * L.grd_sp.y * L.grd_sp.z;
    return L;
}

Layout make_layout(const Geo &g, const Launch &L, int solver, int precision)
{
    Layout y;
    y.fp32_arrays = precision == HOSC_FP32_REFINED ? 15 : 0;
    y.alt_arrays = precision == HOSC_FP32_REFINED ? 4 : 0;
    y.n3 = g.n3;
    y.cs = g.cs;
    y.bicg_arrays = solver == HOSC_SOLVER_SOR ? 0 : 28;
    const size_t recs = std::max({L.nb_int * 8, L.nb_sw * 4, L.nb_face * 2, L.nb_all * 3, L.nb_bc * 8, L.nb_sp * 4});
    y.partial = recs;
    size_t b = 0;
    b += y.natural_arrays * align_up(g.n3 * sizeof(double));
    b += (y.colour_arrays + y.bicg_arrays + y.alt_arrays) * align_up(2 * g.cs * sizeof(double));
    b += y.fp32_arrays * align_up(2 * g.cs * sizeof(float));
    b += 4 * align_up(recs * sizeof(double));                 // partial buffers: red / black half, last and first sweep
    b += align_up(kRed * sizeof(double));                      // reduction outputs
    b += align_up((size_t)g.N * sizeof(double));               // Simpson weights
    b += 2 * align_up((size_t)g.N * g.N * sizeof(double));     // Nu_local hot / cold
    b += 3 * align_up((size_t)g.N * sizeof(double));           // Nu_avg hot / cold, hot-wall row maxima
    b += align_up(8 * sizeof(double));                         // Nu scalars
    b += align_up(32 * sizeof(double));                        // BiCGSTAB scalars
    y.total_bytes = b;
    return y;
}

const char *check_params(const hosc_params *p)
{
    if (!p) return "params is NULL";
    if (p->N < 5 || p->N > 1025) return "N must be in [5, 1025]";
    if (p->precision != HOSC_FP64 && p->precision != HOSC_FP32_REFINED) return "unknown precision";
    if (!(p->Ra >= 0.0) || !std::isfinite(p->Ra)) return "Ra must be finite and >= 0";
    if (!(p->Pr > 0.0) || !std::isfinite(p->Pr)) return "Pr must be finite and > 0";
    if (!(p->n_pl > 0.0 && p->n_pl <= 2.0)) return "n_pl must be in (0, 2]";
    if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return "dt must be finite and > 0";
    if (!(p->lambda >= 0.0) || !std::isfinite(p->lambda)) return "lambda must be finite and >= 0";
    if (!std::isfinite(p->div_tol)) return "div_tol must be finite";
    if (!(p->solve_rtol > 0.0 && p->solve_rtol < 1.0)) return "solve_rtol must be in (0, 1)";
    if (p->solve_maxit < 1) return "solve_maxit must be >= 1";
    if (p->check_every < 0) return "check_every must be >= 0";
    if (!(p->omega >= 0.0 && p->omega < 2.0)) return "omega must be 0 (adaptive) or in (0, 2)";
    if (p->solver < HOSC_SOLVER_AUTO || p->solver > HOSC_SOLVER_BICGSTAB) return "unknown solver";
    if (p->p_iters < 0 || p->p_iters > 64) return "p_iters must be in [0, 64]";
    if (!(p->i2_floor > 0.0) || !std::isfinite(p->i2_floor)) return "i2_floor must be finite and > 0";
    if (!(p->phi >= 0.0) || !std::isfinite(p->phi)) return "phi must be finite and >= 0";
    if (!(p->eta_relax > 0.0 && p->eta_relax <= 1.0)) return "eta_relax must be in (0, 1]";
    if (!std::isfinite(p->theta_hot) || !std::isfinite(p->theta_cold) || !std::isfinite(p->theta_ref))
        return "wall and reference temperatures must be finite";
    return nullptr;
}

// Composite Simpson weights on N equally spaced nodes of [0, 1] (Simpson's 3/8 rule
// on the last three intervals when N-1 is odd).
std::vector<double> simpson(int N)
{
    std::vector<double> w(N, 0.0);
    const double h = 1.0 / (N - 1);
    const int nint = N - 1;
    const int n13 = (nint % 2 == 0) ? nint : nint - 3;
    for (int q = 0; q < n13; q += 2) {
        w[q] += h / 3.0;
        w[q + 1] += 4.0 * h / 3.0;
        w[q + 2] += h / 3.0;
    }
    if (n13 != nint) {
        const int q = n13;
        w[q] += 3.0 * h / 8.0;
        w[q + 1] += 9.0 * h / 8.0;
        w[q + 2] += 9.0 * h / 8.0;
        w[q + 3] += 3.0 * h / 8.0;
    }
    return w;
}

// SplitMix64 (Steele, Lea & Flood 2014): output k of the stream seeded with s.
inline uint64_t splitmix64(uint64_t s, uint64_t k)
{
    uint64_t z = s + (k + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

std::string g_create_error;

}  // namespace

struct hosc_solver {
    hosc_params P;
    Geo g;
    Phys ph;
    Launch L;
    Layout Y;
    hipStream_t st = nullptr;
    int device = 0;
    // natural layout
    double *u, *v, *w, *T, *p, *u2, *v2, *w2, *eta, *etap, *E[3], *Ep[3], *dbg;
    double *u_first = nullptr;      // the buffer u had at creation (level parity of the swapped pointers)
    // colour layout
    double *ms, *ma[3], *mb[3], *md[3], *ta[3], *tb, *td;
    double *partR, *partB, *partR0, *partB0, *red, *wq, *nuh, *nuc, *avh, *avc, *mxh, *nuout;
    // BiCGSTAB vectors (4 systems) and scalars
    double *br[4], *brh[4], *bp[4], *bpn[4], *bv[4], *bvn[4], *bt[4];
    double *bsc;
    int64_t bicg_until[2] = {-1, -1};   // auto mode: use BiCGSTAB for the group until this step
    // precision mode: FP32 copies of the rows, FP32 residuals and corrections of the
    // inner solves
    bool fp32 = false;
    float *fms = nullptr, *fma[3] = {nullptr, nullptr, nullptr}, *fta[3] = {nullptr, nullptr, nullptr};
    float *fr[4] = {nullptr, nullptr, nullptr, nullptr}, *fe[4] = {nullptr, nullptr, nullptr, nullptr};
    double *dalt[4] = {nullptr, nullptr, nullptr, nullptr};   // second increment buffers of the refinement
    double *hbuf = nullptr;   // pinned host staging for scalars
    // mapped, coherent pinned host mirror of the reduction block red[0..kRed): the
    // reductions whose results the host reads write them here too (hmir_dev is its
    // device address), so a convergence check needs no device-to-host copy
    double *hmir = nullptr, *hmir_dev = nullptr;
    int64_t step = 0;
    bool first = true;
    bool has_state = false;
    int sticky = HOSC_OK;
    int last_sweeps[2] = {0, 0};
    // precision mode: sweeps that sufficed in the first inner solve of a step and in
    // the later ones (their right-hand sides differ by decades), and which of the two
    // the next inner solve plans from
    int inner_sweeps[2][2] = {{0, 0}, {0, 0}};
    int inner_slot = 0;
    int last_bicg[2] = {0, 0};
    double om[2] = {1.0, 1.0};          // SOR relaxation of each group (adaptive when P.omega == 0)
    int64_t seeded_at = -1;             // step whose dominance bound was last applied to om
    bool eta_ready = false;             // eta of level n already computed (by the previous step's diagnostics)
    bool diag_valid = false;            // diag holds the diagnostics of level n
    hosc_diag diag{};
    std::string err;
    // kernel timing
    bool prof = false;
    std::vector<hipEvent_t> ev;     // pairs (start, stop)
    std::vector<double> ev_bytes;   // algorithmic bytes of each timed launch
    std::vector<int> ev_kind;       // 0 sweep, 1 assemble, 2 BiCGSTAB phase
    std::vector<int> ev_count;      // kernel launches between the two events
    int ev_used = 0;
    hosc_perf perf{};
};

namespace {

hosc_status fail(hosc_solver *s, hosc_status st, const std::string &msg)
{
    if (s) s->err = msg;
    else g_create_error = msg;
    return st;
}

#define HIPCHK(s, call)                                                                            \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail((s), HOSC_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));    \
    } while (0)

// Wait for a stream by polling.  The convergence checks sit on the critical path
// between batches of kernels; a polling wait resumes the host within microseconds
// of the last kernel, a blocking one can take tens.  Every kernel terminates, so
// the loop ends.
hipError_t wait_stream(hipStream_t st)
{
    for (;;) {
        const hipError_t e = hipStreamQuery(st);
        if (e != hipErrorNotReady) return e;
    }
}

hosc_status launch_check(hosc_solver *s, const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(s, HOSC_E_DEVICE, std::string("launch of ") + what + ": " + hipGetErrorString(e));
    return HOSC_OK;
}

void carve(hosc_solver *s, char *base)
{
    const size_t nat = align_up(s->g.n3 * sizeof(double));
    const size_t col = align_up(2 * s->g.cs * sizeof(double));
    char *q = base;
    auto take = [&](size_t bytes) {
        double *r = reinterpret_cast<double *>(q);
        q += bytes;
        return r;
    };
    s->u = take(nat); s->v = take(nat); s->w = take(nat); s->T = take(nat); s->p = take(nat);
    s->u_first = s->u;
    s->u2 = take(nat); s->v2 = take(nat); s->w2 = take(nat);
    s->eta = take(nat); s->etap = take(nat);
    for (int d = 0; d < 3; ++d) s->E[d] = take(nat);
    for (int d = 0; d < 3; ++d) s->Ep[d] = take(nat);
    s->dbg = take(nat);
    s->ms = take(col);
    for (int d = 0; d < 3; ++d) s->ma[d] = take(col);
    for (int d = 0; d < 3; ++d) s->mb[d] = take(col);
    for (int d = 0; d < 3; ++d) s->md[d] = take(col);
    for (int d = 0; d < 3; ++d) s->ta[d] = take(col);
    s->tb = take(col);
    s->td = take(col);
    const size_t pb = align_up(s->Y.partial * sizeof(double));
    s->partR = take(pb);
    s->partB = take(pb);
    s->partR0 = take(pb);
    s->partB0 = take(pb);
    s->red = take(align_up(kRed * sizeof(double)));
    s->wq = take(align_up((size_t)s->g.N * sizeof(double)));
    s->nuh = take(align_up((size_t)s->g.N * s->g.N * sizeof(double)));
    s->nuc = take(align_up((size_t)s->g.N * s->g.N * sizeof(double)));
    s->avh = take(align_up((size_t)s->g.N * sizeof(double)));
    s->avc = take(align_up((size_t)s->g.N * sizeof(double)));
    s->mxh = take(align_up((size_t)s->g.N * sizeof(double)));
    s->nuout = take(align_up(8 * sizeof(double)));
    s->bsc = take(align_up(32 * sizeof(double)));
    for (int f = 0; f < 4; ++f) s->br[f] = s->brh[f] = s->bp[f] = s->bpn[f] = s->bv[f] = s->bvn[f] = s->bt[f] = nullptr;
    s->fp32 = s->Y.fp32_arrays > 0;
    if (s->fp32) {
        const size_t fcol = align_up(2 * s->g.cs * sizeof(float));
        s->fms = reinterpret_cast<float *>(take(fcol));
        for (int d = 0; d < 3; ++d) s->fma[d] = reinterpret_cast<float *>(take(fcol));
        for (int d = 0; d < 3; ++d) s->fta[d] = reinterpret_cast<float *>(take(fcol));
        for (int f = 0; f < 4; ++f) s->fr[f] = reinterpret_cast<float *>(take(fcol));
        for (int f = 0; f < 4; ++f) s->fe[f] = reinterpret_cast<float *>(take(fcol));
        for (int f = 0; f < 4; ++f) s->dalt[f] = take(col);
    }
    if (s->Y.bicg_arrays)
        for (int f = 0; f < 4; ++f) {
            s->br[f] = take(col); s->brh[f] = take(col); s->bp[f] = take(col); s->bpn[f] = take(col);
            s->bv[f] = take(col); s->bvn[f] = take(col); s->bt[f] = take(col);
        }
}

constexpr int kEvPairs = 512;

// Algorithmic bytes of one half-sweep launch (see hosc_perf in hosc.h).
double sweep_bytes(const Geo &g, int mask, size_t elem = sizeof(double))
{
    const double nodes = 0.5 * (double)(g.N - 2) * (g.N - 2) * (g.N - 2);
    double per = 0.0;
    int nf = 0;     // momentum fields swept
    for (int f = 0; f < 3; ++f) nf += ((mask >> (2 + f)) & 1) ? 0 : 1;
    if (mask & 1) per += (4 + 4 * nf) * elem;   // row 4; per field rhs 1, own 1 read + 1 write, other colour 1
    if (mask & 2) per += (4 + 1 + 1 + 1) * elem;   // row 3 + rhs 1, own 1 + 1, other colour 1
    return nodes * per;
}

// Algorithmic bytes of one refinement pass (both colours, every interior node):
// FP64 rows and right-hand sides, FP64 increment, FP32 residual written, and for
// the systems in emask the FP32 correction read and the folded FP64 increment
// written.  The neighbours are the other colour's entries of the same pass.
double refine_bytes(const Geo &g, int mask, int emask)
{
    const double nodes = (double)(g.N - 2) * (g.N - 2) * (g.N - 2);
    double per = 0.0;
    if (mask & 1) per += 4 * 8;
    if (mask & 2) per += 3 * 8;
    for (int f = 0; f < 4; ++f) {
        if (!((f < 3) ? (mask & 1) : (mask & 2))) continue;
        per += 8 + 8 + 4 + (((emask >> f) & 1) ? 4 + 8 : 0);
    }
    return nodes * per;
}

// Algorithmic bytes of the assembly: 8 level-n fields and 7 level n-1 fields read,
// 11 row arrays written, per interior node.
double assemble_bytes(const Geo &g)
{
    return (double)(g.N - 2) * (g.N - 2) * (g.N - 2) * (15 + 11) * sizeof(double);
}

// Fold the recorded event pairs into the counters.  Called only when the pairs are
// used up, when the counters are read and when timing is switched: reading the
// elapsed times after each convergence check would put host work between the
// check and the next launch (about 1% of a 129^3 step).
hosc_status harvest_events(hosc_solver *s)
{
    if (!s->prof || s->ev_used == 0) return HOSC_OK;
    HIPCHK(s, hipEventSynchronize(s->ev[2 * (s->ev_used - 1) + 1]));
    for (int q = 0; q < s->ev_used; ++q) {
        float ms = 0.0f;
        HIPCHK(s, hipEventElapsedTime(&ms, s->ev[2 * q], s->ev[2 * q + 1]));
        if (s->ev_kind[q] == 0) {
            s->perf.sweep_launches += s->ev_count[q];
            s->perf.sweep_ms += ms;
            s->perf.sweep_bytes += s->ev_bytes[q];
        } else if (s->ev_kind[q] == 1) {
            s->perf.assemble_launches += 1;
            s->perf.assemble_ms += ms;
            s->perf.assemble_bytes += s->ev_bytes[q];
        } else if (s->ev_kind[q] == 2) {
            s->perf.bicg_launches += s->ev_count[q];
            s->perf.bicg_ms += ms;
            s->perf.bicg_bytes += s->ev_bytes[q];
        } else {
            s->perf.refine_launches += s->ev_count[q];
            s->perf.refine_ms += ms;
            s->perf.refine_bytes += s->ev_bytes[q];
        }
    }
    s->ev_used = 0;
    return HOSC_OK;
}

// Bracket the next launch with events when timing is on.
hosc_status timed_begin(hosc_solver *s)
{
    if (!s->prof) return HOSC_OK;
    if (s->ev_used == kEvPairs) {
        hosc_status r = harvest_events(s);
        if (r) return r;
    }
    HIPCHK(s, hipEventRecord(s->ev[2 * s->ev_used], s->st));
    return HOSC_OK;
}
hosc_status timed_end(hosc_solver *s, int kind, double bytes, int count = 1)
{
    if (!s->prof) return HOSC_OK;
    HIPCHK(s, hipEventRecord(s->ev[2 * s->ev_used + 1], s->st));
    s->ev_kind[s->ev_used] = kind;
    s->ev_bytes[s->ev_used] = bytes;
    s->ev_count[s->ev_used] = count;
    s->ev_used += 1;
    return HOSC_OK;
}

// Zero the increments and every BiCGSTAB vector.  The kernels only ever write
// interior entries, so the wall entries of these colour arrays stay zero: the
// Dirichlet walls of the increment systems.
hosc_status zero_colour_increments(hosc_solver *s)
{
    const size_t b = 2 * s->g.cs * sizeof(double);
    for (int d = 0; d < 3; ++d) HIPCHK(s, hipMemsetAsync(s->md[d], 0, b, s->st));
    HIPCHK(s, hipMemsetAsync(s->td, 0, b, s->st));
    if (s->Y.bicg_arrays)
        for (int f = 0; f < 4; ++f) {
            double *v[7] = {s->br[f], s->brh[f], s->bp[f], s->bpn[f], s->bv[f], s->bvn[f], s->bt[f]};
            for (double *x : v) HIPCHK(s, hipMemsetAsync(x, 0, b, s->st));
        }
    if (s->fp32)
        for (int f = 0; f < 4; ++f) {
            HIPCHK(s, hipMemsetAsync(s->fr[f], 0, 2 * s->g.cs * sizeof(float), s->st));
            HIPCHK(s, hipMemsetAsync(s->fe[f], 0, 2 * s->g.cs * sizeof(float), s->st));
            HIPCHK(s, hipMemsetAsync(s->dalt[f], 0, b, s->st));
        }
    return HOSC_OK;
}

// Boundary conditions on level n (device).
hosc_status impose_bc(hosc_solver *s)
{
    k_zero_walls<<<s->L.grd_face, s->L.blk_face, 0, s->st>>>(s->g, s->u, s->v, s->w);
    k_theta_walls<<<s->L.grd_face, s->L.blk_face, 0, s->st>>>(s->g, s->ph, s->T, s->partR);
    k_p_walls<<<s->L.grd_face, s->L.blk_face, 0, s->st>>>(s->g, s->p);
    return launch_check(s, "boundary conditions");
}

hosc_status reset_state(hosc_solver *s)
{
    hosc_status r = zero_colour_increments(s);
    if (r) return r;
    s->step = 0;
    s->first = true;
    s->has_state = true;
    s->sticky = HOSC_OK;
    s->last_sweeps[0] = s->last_sweeps[1] = 0;
    for (auto &h : s->inner_sweeps) h[0] = h[1] = 0;
    s->last_bicg[0] = s->last_bicg[1] = 0;
    s->bicg_until[0] = s->bicg_until[1] = -1;
    s->om[0] = s->om[1] = s->P.omega > 0.0 ? s->P.omega : 1.0;
    s->seeded_at = -1;
    s->eta_ready = false;
    s->diag_valid = false;
    HIPCHK(s, hipStreamSynchronize(s->st));
    return HOSC_OK;
}

// eta and E* at level n; on the first step level n-1 := level n.
hosc_status stage_sources(hosc_solver *s, bool consume_first)
{
    if (!s->eta_ready) k_eta<<<s->L.grd_all, s->L.blk_all, 0, s->st>>>(s->g, s->ph, s->u, s->v, s->w, s->eta);
    k_estar<<<s->L.grd_all, s->L.blk_all, 0, s->st>>>(s->g, s->ph, s->u, s->v, s->w, s->T, s->p, s->eta, s->E[0],
                                                       s->E[1], s->E[2]);
    hosc_status r = launch_check(s, "eta/estar");
    if (r) return r;
    if (s->first) {
        // level n-1 := level n for u, v, w, eta and E*, in two copy launches (each
        // natural array is 256-byte aligned and padded, so an odd n3 rounds up to
        // whole 16-byte pairs inside its region)
        const double *src[7] = {s->u, s->v, s->w, s->eta, s->E[0], s->E[1], s->E[2]};
        double *dst[7] = {s->u2, s->v2, s->w2, s->etap, s->Ep[0], s->Ep[1], s->Ep[2]};
        const size_t n = (s->g.n3 + 1) / 2;
        const unsigned blocks = (unsigned)std::min<size_t>(2048, (n + 255) / 256);
        for (int a0 = 0; a0 < 7; a0 += 4) {
            Copies4 cp{};
            for (int a = a0; a < std::min(7, a0 + 4); ++a) {
                cp.src[cp.count] = reinterpret_cast<const double2 *>(src[a]);
                cp.dst[cp.count] = reinterpret_cast<double2 *>(dst[a]);
                cp.count += 1;
            }
            k_copy4<<<blocks, 256, 0, s->st>>>(cp, n);
        }
        r = launch_check(s, "level copies");
        if (r) return r;
        if (consume_first) s->first = false;
    }
    return HOSC_OK;
}

// FP64 solve: the rows, right-hand sides and increments of the step
SweepArgs<double> sweep_args(hosc_solver *s)
{
    SweepArgs<double> a;
    a.ms = s->ms;
    for (int d = 0; d < 3; ++d) {
        a.ma[d] = s->ma[d];
        a.mb[d] = s->mb[d];
        a.md[d] = s->md[d];
        a.ta[d] = s->ta[d];
    }
    a.tb = s->tb;
    a.td = s->td;
    return a;
}

// FP32 inner solve of the precision mode: FP32 rows, residuals and corrections
SweepArgs<float> sweep_args_fp32(hosc_solver *s)
{
    SweepArgs<float> a;
    a.ms = s->fms;
    for (int d = 0; d < 3; ++d) {
        a.ma[d] = s->fma[d];
        a.mb[d] = s->fr[d];
        a.md[d] = s->fe[d];
        a.ta[d] = s->fta[d];
    }
    a.tb = s->fr[3];
    a.td = s->fe[3];
    return a;
}

// Launch up to four reductions in one kernel (jobs in order; n <= 4).
struct Reductions {
    ReduceJobs4 r{};
    int n = 0;
    Reductions &add(const double *part, size_t nb, int nc, int op, double *out, double *out_host = nullptr)
    {
        ReduceJob &j = r.j[n++];
        j.part = part;
        j.nb = (int)nb;
        j.nc = nc;
        j.op = op;
        j.out = out;
        j.out_host = out_host;
        j.pad = 0;
        return *this;
    }
    void launch(hipStream_t st) const { k_reduce4<<<n, 1024, 0, st>>>(r); }
};

// Device address of the host mirror of red[i] for out = red + i.
double *mir(const hosc_solver *s, const double *out) { return s->hmir_dev + (out - s->red); }

// Algorithmic bytes of one BiCGSTAB phase launch over both colours.
double bicg_bytes(const Geo &g, int phase, int mask)
{
    const double nodes = (double)(g.N - 2) * (g.N - 2) * (g.N - 2);
    // per system: vectors touched (reads + writes); rows counted once per matrix
    static const int vec[4] = {6, 5, 3, 8};   // phase 0: b, x | r, rh, p, v;  1: r, p, v, rh | pn, vn;  2: r, vn | t;  3: r, vn, x, pn, t, rh | x, r
    static const int rows[4] = {1, 1, 1, 0};
    double per = 0.0;
    if (mask & 1) per += 3 * vec[phase] + rows[phase] * 4;
    if (mask & 2) per += vec[phase] + rows[phase] * 3;
    return nodes * per * sizeof(double);
}

struct SolveOut {
    double relres[4] = {0, 0, 0, 0};
    double dominance[2] = {0, 0};
    int sweeps[2] = {0, 0};
    int bicg[2] = {0, 0};
    int corrections = 0;    // pressure corrections made between the momentum solves of the step
};

hosc_status zero_group(hosc_solver *s, int group)
{
    const size_t b = 2 * s->g.cs * sizeof(double);
    if (group == 0)
        for (int f = 0; f < 3; ++f) HIPCHK(s, hipMemsetAsync(s->md[f], 0, b, s->st));
    else
        HIPCHK(s, hipMemsetAsync(s->td, 0, b, s->st));
    return HOSC_OK;
}

// Red-black SOR on the groups in `mask` (1 momentum, 2 energy) until each meets
// ||r|| <= rtol ||b|| (scaled rows).  One sweep = red half then black half; the sums
// of squared pre-update residuals of the black half and (1-omega)^2 times those of
// the red half give the residual of the state between the two halves, so
// convergence is known without an extra pass.  Each group plans its own number of
// sweeps per batch (from its count at the previous step, then from the measured
// contraction rate); a launch updates only the groups still inside their plan.  In
// auto mode a group whose residual grows or stalls is returned in *failed.
// Young's relation for a consistently ordered matrix (red-black ordering of a
// 7-point stencil is one): an SOR contraction lam at relaxation w gives the
// Jacobi radius mu^2 = (lam + w - 1)^2 / (lam w^2) and the optimum
// w = 2 / (1 + sqrt(1 - mu^2)).  Used, damped and clamped, to adapt w per group.
double young_omega(double lam, double w)
{
    if (!(lam > 0.0 && lam < 1.0)) return w;
    const double mu2 = std::min(0.999, (lam + w - 1.0) * (lam + w - 1.0) / (lam * w * w));
    return 2.0 / (1.0 + std::sqrt(1.0 - mu2));
}

// State of one red-black SOR solve between convergence checks.  The same control
// drives the single-cavity solve and the batched solve of many cavities, so a
// cavity takes the same decisions (sweep plans, relaxation, stopping) either way.
struct SorCtl {
    int active = 0, failed = 0, batch = 0, soft_cap = 0;
    int skip = 0;       // momentum fields with a zero right-hand side (bits 0..2): not swept
    bool inner = false, adapt = false, autom = false;
    bool zero_start = false;    // the first sweep starts from the zero increment without reading it
    double rtol = 0.0;
    double ref[2] = {-1.0, -1.0};
    int ref_at[2] = {0, 0}, plan[2] = {0, 0}, swept[2] = {0, 0}, first_plan[2] = {0, 0};
    int *hist = nullptr;        // sweep history this solve plans from and updates
};

// inner solves of the refinement: at most 200 sweeps, and no relaxation update
// from a first batch (a short batch that starts from zero measures the start-up
// transient, not the asymptotic contraction Young's relation needs)
// Momentum fields with ||b|| = 0 have the zero increment: the sweeps leave them
// out (their increments are zeroed when the group converges).
void sor_skip(SorCtl &c, const double bn2[4])
{
    c.skip = 0;
    if (bn2[0] >= 0.0)
        for (int f = 0; f < 3; ++f)
            if (bn2[f] == 0.0) c.skip |= 1 << f;
}

void sor_begin(hosc_solver *s, SorCtl &c, int mask, double rtol, bool inner)
{
    c = SorCtl();
    c.active = mask;
    c.rtol = rtol;
    c.inner = inner;
    c.zero_start = inner;
    c.soft_cap = inner ? 200 : 0;
    c.adapt = s->P.omega == 0.0;
    c.autom = s->P.solver == HOSC_SOLVER_AUTO;
    c.hist = inner ? s->inner_sweeps[s->inner_slot] : s->last_sweeps;
    for (int grp = 0; grp < 2; ++grp)
        c.plan[grp] = s->P.check_every > 0 ? s->P.check_every : std::max(2, c.hist[grp]);
    c.first_plan[0] = c.plan[0];
    c.first_plan[1] = c.plan[1];
}

// The dominance monitor of this step's assembly (dom = red[44..45]) is a
// Gershgorin bound mu on the Jacobi radius; the relaxation it implies,
// 2 / (1 + sqrt(1 - mu^2)), seeds the first step after a state was set and caps
// the adapted relaxation at every later step, before the first sweep.
// A group whose relaxation the cap lowers by more than 0.05 halves its first batch:
// the sweep count it inherited was measured at the old relaxation.
bool sor_wants_seed(const hosc_solver *s, const SorCtl &c) { return c.adapt && s->seeded_at != s->step; }
void sor_seed(hosc_solver *s, SorCtl &c, const double *dom)
{
    s->seeded_at = s->step;
    for (int grp = 0; grp < 2; ++grp) {
        const double mu = std::min(0.98, dom[grp]);
        if (!(mu > 0.0 && std::isfinite(mu))) continue;
        const double w = 2.0 / (1.0 + std::sqrt(1.0 - mu * mu));
        // sweeps the new relaxation needs from a unit residual (contraction w - 1)
        const int pred = w > 1.0 ? (int)std::ceil(std::log(c.rtol) / std::log(w - 1.0)) : c.plan[grp];
        if (s->step == 0) {
            s->om[grp] = w;
            if (s->P.check_every == 0) c.plan[grp] = std::max(c.plan[grp], std::min(256, pred));
        } else if (w < s->om[grp]) {
            if (s->om[grp] - w > 0.05 && s->P.check_every == 0)
                c.plan[grp] = std::max(2, std::min(c.plan[grp] / 2, pred));
            s->om[grp] = w;
        }
        c.first_plan[grp] = c.plan[grp];
    }
}

// Mask and store flags of sweep q of the current batch.
void sor_sweep_flags(const SorCtl &c, int q, int &m, unsigned &store, unsigned &store0)
{
    static const unsigned kStore[2] = {0x7u, 0x8u};   // residual components of each group
    m = 0;
    store = store0 = 0;
    for (int grp = 0; grp < 2; ++grp) {
        if (!(c.active & (1 << grp)) || q >= c.plan[grp]) continue;
        m |= grp == 0 ? 1 | (c.skip << 2) : 2;
        if (c.zero_start && c.batch == 0 && q == 0) m |= 32;
        if (q == c.plan[grp] - 1) store |= kStore[grp];
        if (q == 0 && c.plan[grp] > 1) store0 |= kStore[grp];
    }
}
int sor_batch_sweeps(const SorCtl &c)
{
    int nsw = 0;
    for (int grp = 0; grp < 2; ++grp)
        if (c.active & (1 << grp)) nsw = std::max(nsw, c.plan[grp]);
    return nsw;
}

// Decisions after a batch of sweeps, from the reduction block hb (the cavity's
// red[0..47]: ||b/C||^2 at 0..3, last-sweep partial sums red/black at 4..11,
// first-sweep sums at 32..39, dominance at 44..45).
template <typename TM>
hosc_status sor_decide(hosc_solver *s, SorCtl &c, const double *hb, double bn2[4], SolveOut &o,
                       const SweepArgs<TM> &a)
{
    o.dominance[0] = hb[44];
    o.dominance[1] = hb[45];
    if (bn2[0] < 0.0) {
        for (int f = 0; f < 4; ++f) bn2[f] = hb[f];
        for (int f = 0; f < 4; ++f)
            if (!std::isfinite(bn2[f])) return fail(s, HOSC_E_NONFINITE, "non-finite right-hand side");
    }
    const double rtol = c.rtol;
    for (int grp = 0; grp < 2; ++grp) {
        if (!(c.active & (1 << grp))) continue;
        o.sweeps[grp] += c.plan[grp];
        c.swept[grp] += c.plan[grp];
        const int done = c.swept[grp];     // sweeps of this call (o.sweeps also counts earlier calls of the step)
        const int f0 = grp == 0 ? 0 : 3, f1 = grp == 0 ? 3 : 4;
        const double om = s->om[grp];
        bool conv = true, finite = true;
        double worst = 0.0, worst0 = 0.0;
        for (int f = f0; f < f1; ++f) {
            const double r2 = hb[8 + f] + (1.0 - om) * (1.0 - om) * hb[4 + f];
            const double r20 = hb[36 + f] + (1.0 - om) * (1.0 - om) * hb[32 + f];
            if (!std::isfinite(r2)) finite = false;
            const double rel = bn2[f] > 0.0 ? std::sqrt(r2 / bn2[f]) : 0.0;
            o.relres[f] = rel;
            worst = std::max(worst, rel);
            if (bn2[f] > 0.0) worst0 = std::max(worst0, std::sqrt(r20 / bn2[f]));
            if (!(bn2[f] == 0.0 || std::sqrt(r2) <= rtol * std::sqrt(bn2[f]))) conv = false;
        }
        // contraction per sweep inside this batch (first vs last sweep)
        double rate = -1.0;
        if (finite && c.plan[grp] > 1 && worst0 > 0.0 && worst > 0.0 && worst < worst0)
            rate = std::pow(worst / worst0, 1.0 / (double)(c.plan[grp] - 1));
        if (c.adapt && rate > 0.0 && rate < 1.0 && c.plan[grp] >= 4 && !(c.inner && c.batch == 0)) {
            // below the optimum the contraction exceeds w - 1 and Young's relation
            // gives the optimum; at or past it the contraction is about w - 1: back off
            // by a fraction of the over-relaxation
            const double w = s->om[grp];
            double wn = (w > 1.05 && rate < (w - 1.0) + 0.02) ? 1.0 + 0.7 * (w - 1.0) : young_omega(rate, w);
            wn = std::min(1.9, std::max(1.0, wn));
            s->om[grp] = w + 0.5 * (wn - w);
        }
        if (finite && conv) {
            for (int f = f0; f < f1; ++f)
                if (bn2[f] == 0.0) {
                    const size_t b = 2 * s->g.cs * sizeof(TM);
                    HIPCHK(s, hipMemsetAsync(f < 3 ? a.md[f] : a.td, 0, b, s->st));
                }
            // sweeps that would have sufficed, for the next step's plan: from the
            // measured rate when there is one; a first batch that converged
            // without a usable rate halves the plan
            int suff = done == c.first_plan[grp] ? std::max(1, done / 2) : done;
            if (rate > 0.0 && rate < 1.0 && worst > 0.0)    // r_done / r_needed = rate^(done - needed)
                suff = done - (int)std::floor(std::log(worst / rtol) / std::log(rate));
            c.hist[grp] = std::max(1, std::min(done, suff));
            c.active &= ~(1 << grp);
            continue;
        }
        // divergence: not finite or grown 2x over the reference; stall: less than a
        // 2x reduction over 100 sweeps
        const bool diverged = !finite || (c.ref[grp] >= 0.0 && worst > 2.0 * c.ref[grp])
                              || (rate < 0.0 && worst > 2.0 * worst0 && worst0 > 0.0);
        const bool stalled = c.ref[grp] >= 0.0 && done - c.ref_at[grp] >= 100 && worst > 0.5 * c.ref[grp];
        if (c.soft_cap > 0 && done >= c.soft_cap && !diverged) {
            // inner solve of the refinement: stop here, the outer pass takes what it has
            c.active &= ~(1 << grp);
            continue;
        }
        if (diverged || stalled || done >= s->P.solve_maxit) {
            if (c.autom) {
                c.failed |= 1 << grp;
                c.active &= ~(1 << grp);
                continue;
            }
            if (!finite) return fail(s, HOSC_E_NONFINITE, "non-finite residual in the implicit solve");
            if (done >= s->P.solve_maxit)
                return fail(s, HOSC_E_NOCONV, "implicit solve did not converge within solve_maxit sweeps");
        }
        if (c.ref[grp] < 0.0 || done - c.ref_at[grp] >= 100) {
            c.ref[grp] = worst;
            c.ref_at[grp] = done;
        }
        int next = std::max(2, std::min(done, 64));
        if (rate > 0.0 && rate < 1.0)
            next = (int)std::min(256.0, std::max(2.0, std::ceil(std::log(rtol / worst) / std::log(rate)) + 1.0));
        // at most double the sweeps of this solve: the contraction of a short batch
        // still carries the start-up transient (over-relaxed red-black SOR decays
        // like k (w-1)^k before it settles) and overstates what is left
        if (!c.inner) next = std::min(next, std::max(4, done));
        c.plan[grp] = s->P.check_every > 0 ? s->P.check_every : next;
        c.plan[grp] = std::min(c.plan[grp], std::max(1, s->P.solve_maxit - done));
    }
    c.batch += 1;
    return HOSC_OK;
}

// the constant s/C of the scaled energy rows
double theta_st(const hosc_solver *s)
{
    const double ct = s->g.h2 / 12.0 - s->P.dt / 2.0;
    const double Ct = 1.0 - 6.0 * ct * s->g.invh2;
    return (ct * s->g.invh2) / Ct;
}

// Single-cavity solve: batches of sweeps on the solver's stream, a host check after each.
template <typename TM>
hosc_status run_sor(hosc_solver *s, int mask, double bn2[4], SolveOut &o, int *failed, SweepArgs<TM> a, double rtol,
                    bool inner = false)
{
    const double st = theta_st(s);
    SorCtl c;
    sor_begin(s, c, mask, rtol, inner);
    *failed = 0;
    if (sor_wants_seed(s, c)) {
        HIPCHK(s, wait_stream(s->st));
        sor_seed(s, c, s->hmir + 44);
        if (bn2[0] < 0.0) {
            for (int f = 0; f < 4; ++f) bn2[f] = s->hmir[f];
            for (int f = 0; f < 4; ++f)
                if (!std::isfinite(bn2[f])) return fail(s, HOSC_E_NONFINITE, "non-finite right-hand side");
        }
    }
    sor_skip(c, bn2);
    while (c.active) {
        const int nsw = sor_batch_sweeps(c);
        hosc_status r = timed_begin(s);
        if (r) return r;
        double bytes = 0.0;
        for (int q = 0; q < nsw; ++q) {
            int m;
            unsigned store, store0;
            sor_sweep_flags(c, q, m, store, store0);
            bytes += 2.0 * sweep_bytes(s->g, m, sizeof(TM));
            for (int colour = 0; colour < 2; ++colour)
                k_sweep<TM, TM><<<s->L.grd_sp, s->L.blk_sp, 0, s->st>>>(
                    s->g, colour, m, (TM)s->om[0], (TM)s->om[1], (TM)st, a, colour ? s->partB : s->partR, store,
                    colour ? s->partB0 : s->partR0, store0);
        }
        r = timed_end(s, 0, bytes, 2 * nsw);
        if (r) return r;
        r = launch_check(s, "sweep");
        if (r) return r;
        Reductions()
            .add(s->partR, s->L.nb_sp, 4, 0, s->red + 4, mir(s, s->red + 4))
            .add(s->partB, s->L.nb_sp, 4, 0, s->red + 8, mir(s, s->red + 8))
            .add(s->partR0, s->L.nb_sp, 4, 0, s->red + 32, mir(s, s->red + 32))
            .add(s->partB0, s->L.nb_sp, 4, 0, s->red + 36, mir(s, s->red + 36))
            .launch(s->st);
        HIPCHK(s, wait_stream(s->st));
        r = sor_decide<TM>(s, c, s->hmir, bn2, o, a);
        if (r) return r;
    }
    *failed = c.failed;
    return HOSC_OK;
}

template <typename TR>
BicgArgs<TR, double> bicg_args(hosc_solver *s, const TR *ms, const TR *const ma[3], const TR *const ta[3])
{
    BicgArgs<TR, double> a;
    a.ms = ms;
    for (int d = 0; d < 3; ++d) {
        a.ma[d] = ma[d];
        a.mb[d] = s->mb[d];
        a.ta[d] = ta[d];
    }
    a.tb = s->tb;
    for (int f = 0; f < 4; ++f) {
        a.x[f] = f < 3 ? s->md[f] : s->td;
        a.r[f] = s->br[f]; a.rh[f] = s->brh[f]; a.p[f] = s->bp[f]; a.pn[f] = s->bpn[f];
        a.v[f] = s->bv[f]; a.vn[f] = s->bvn[f]; a.t[f] = s->bt[f];
    }
    return a;
}

template <typename TR>
hosc_status bicg_phase(hosc_solver *s, int phase, int mask, double st, const BicgArgs<TR, double> &a)
{
    hosc_status r = timed_begin(s);
    if (r) return r;
    k_bicg<TR, double, double><<<s->L.grd_bc, s->L.blk_sw, 0, s->st>>>(s->g, phase, mask, st, a, s->bsc, s->partR);
    r = timed_end(s, 2, bicg_bytes(s->g, phase, mask));
    if (r) return r;
    k_bicg_scalars<<<1, 1024, 0, s->st>>>(phase, mask, s->partR, (int)s->L.nb_bc, s->bsc);
    return launch_check(s, "bicgstab");
}

// BiCGSTAB (the paper's solver) on the groups in `mask`, from the current
// increments, until the true scaled residual meets the tolerance.
template <typename TR>
hosc_status run_bicg(hosc_solver *s, int mask, double bn2[4], SolveOut &o, BicgArgs<TR, double> a)
{
    if (!mask) return HOSC_OK;
    if (bn2[0] < 0.0) {
        HIPCHK(s, wait_stream(s->st));
        for (int f = 0; f < 4; ++f) bn2[f] = s->hmir[f];
        for (int f = 0; f < 4; ++f)
            if (!std::isfinite(bn2[f])) return fail(s, HOSC_E_NONFINITE, "non-finite right-hand side");
    }
    const double rtol = s->P.solve_rtol;
    const double ct = s->g.h2 / 12.0 - s->P.dt / 2.0;
    const double Ct = 1.0 - 6.0 * ct * s->g.invh2;
    const double st = (ct * s->g.invh2) / Ct;
    int active = mask;
    for (int grp = 0; grp < 2; ++grp) {     // groups with b = 0 have the zero solution
        if (!(active & (1 << grp))) continue;
        const int f0 = grp == 0 ? 0 : 3, f1 = grp == 0 ? 3 : 4;
        bool zero = true;
        for (int f = f0; f < f1; ++f) zero = zero && bn2[f] == 0.0;
        if (zero) {
            hosc_status r = zero_group(s, grp);
            if (r) return r;
            active &= ~(1 << grp);
        }
    }
    if (!active) return HOSC_OK;
    hosc_status r = bicg_phase(s, 0, active, st, a);
    if (r) return r;
    int m = std::max(2, std::max(s->last_bicg[0], s->last_bicg[1]) / 2);
    if (s->P.check_every > 0) m = s->P.check_every;
    // stall guard: a group whose recursive residual has not halved within
    // kBicgStall iterations is reported unconverged at once instead of at solve_maxit
    constexpr int kBicgStall = 400;
    double best[2] = {HUGE_VAL, HUGE_VAL};
    int best_at[2] = {0, 0};
    while (active) {
        for (int q = 0; q < m; ++q) {
            for (int ph = 1; ph <= 3; ++ph) {
                r = bicg_phase(s, ph, active, st, a);
                if (r) return r;
            }
            for (int f = 0; f < 4; ++f) {
                std::swap(a.p[f], a.pn[f]);
                std::swap(a.v[f], a.vn[f]);
            }
        }
        for (int grp = 0; grp < 2; ++grp)
            if (active & (1 << grp)) o.bicg[grp] += m;
        HIPCHK(s, hipMemcpyAsync(s->hbuf, s->bsc, 32 * sizeof(double), hipMemcpyDeviceToHost, s->st));
        HIPCHK(s, wait_stream(s->st));
        // candidates: recursive residual small enough, or breakdown -> recompute the true
        // residual from x (this also restarts the recurrence)
        int recheck = 0;
        for (int grp = 0; grp < 2; ++grp) {
            if (!(active & (1 << grp))) continue;
            const int f0 = grp == 0 ? 0 : 3, f1 = grp == 0 ? 3 : 4;
            bool small = true, broke = false;
            double worst = 0.0;
            for (int f = f0; f < f1; ++f) {
                const double *S = s->hbuf + 8 * f;
                if (!std::isfinite(S[4])) return fail(s, HOSC_E_NONFINITE, "non-finite residual in BiCGSTAB");
                if (S[5] != 0.0) broke = true;
                if (!(bn2[f] == 0.0 || std::sqrt(S[4]) <= rtol * std::sqrt(bn2[f]))) small = false;
                if (bn2[f] > 0.0) worst = std::max(worst, std::sqrt(S[4] / bn2[f]));
            }
            if (worst < 0.5 * best[grp]) {
                best[grp] = worst;
                best_at[grp] = o.bicg[grp];
            } else if (!small && !broke && o.bicg[grp] - best_at[grp] >= kBicgStall) {
                return fail(s, HOSC_E_NOCONV, "BiCGSTAB stalled: the residual did not halve in " +
                                                  std::to_string(kBicgStall) + " iterations");
            }
            if (small || broke) recheck |= 1 << grp;
        }
        if (recheck) {
            r = bicg_phase(s, 0, recheck, st, a);
            if (r) return r;
            HIPCHK(s, hipMemcpyAsync(s->hbuf, s->bsc, 32 * sizeof(double), hipMemcpyDeviceToHost, s->st));
            HIPCHK(s, wait_stream(s->st));
            for (int grp = 0; grp < 2; ++grp) {
                if (!(recheck & (1 << grp))) continue;
                const int f0 = grp == 0 ? 0 : 3, f1 = grp == 0 ? 3 : 4;
                bool conv = true;
                for (int f = f0; f < f1; ++f) {
                    const double rr = s->hbuf[8 * f + 4];
                    o.relres[f] = bn2[f] > 0.0 ? std::sqrt(rr / bn2[f]) : 0.0;
                    if (!(bn2[f] == 0.0 || std::sqrt(rr) <= rtol * std::sqrt(bn2[f]))) conv = false;
                }
                if (conv) active &= ~(1 << grp);
            }
        }
        const int done = std::max(o.bicg[0], o.bicg[1]);
        if (active && done >= s->P.solve_maxit)
            return fail(s, HOSC_E_NOCONV, "BiCGSTAB did not converge within solve_maxit iterations");
    }
    return HOSC_OK;
}

// Solve the momentum (3 right-hand sides) and energy systems of the step.
// Precision mode: iterative refinement.  Each outer pass (one launch over both
// colours) forms the FP64 residual of the scaled FP64 rows at the current iterate
// and folds the FP32 correction of the last inner solve into the FP64 increment;
// converged groups stop, the others solve B e = r for the FP32 correction with
// FP32 red-black sweeps to a relative 1e-5 or what the tolerance still needs.
// Groups whose inner solve fails (auto mode) are returned in *to_bicg.
//
// The fold writes d + e to the other of two FP64 increment buffers (cur / oth
// swap per system); when the solve ends, a system whose increment is in the
// second buffer is copied back, so the rest of the step sees one buffer.
struct RefCtl {
    int active = 0, outer = 0, to_bicg = 0;
    int emask = 0;                  // systems whose FP32 correction is not yet folded
    double *cur[4] = {nullptr, nullptr, nullptr, nullptr}, *oth[4] = {nullptr, nullptr, nullptr, nullptr};
};

double *primary_increment(hosc_solver *s, int f) { return f < 3 ? s->md[f] : s->td; }

void refine_begin(hosc_solver *s, RefCtl &c, int mask)
{
    c = RefCtl();
    c.active = mask;
    for (int f = 0; f < 4; ++f) {
        c.cur[f] = primary_increment(s, f);
        c.oth[f] = s->dalt[f];
    }
}

RefineArgs<double> refine_args(hosc_solver *s, const RefCtl &c)
{
    RefineArgs<double> ra;
    ra.ms = s->ms;
    for (int d = 0; d < 3; ++d) {
        ra.ma[d] = s->ma[d];
        ra.ta[d] = s->ta[d];
        ra.b[d] = s->mb[d];
    }
    ra.b[3] = s->tb;
    for (int f = 0; f < 4; ++f) {
        ra.d[f] = c.cur[f];
        ra.dn[f] = c.oth[f];
        ra.e[f] = s->fe[f];
        ra.r[f] = s->fr[f];
    }
    return ra;
}

// After a pass is launched: the folded systems now live in their other buffer.
void refine_folded(RefCtl &c)
{
    for (int f = 0; f < 4; ++f)
        if (((c.emask >> f) & 1) && (c.active & (f < 3 ? 1 : 2))) std::swap(c.cur[f], c.oth[f]);
    c.emask = 0;
}

// Systems whose increment sits in the second buffer are copied back, in one launch
// (stream order; the colour arrays hold 2 cs doubles, an even count, 256-byte aligned).
hosc_status refine_end(hosc_solver *s, RefCtl &c, hipStream_t st)
{
    Copies4 cp{};
    for (int f = 0; f < 4; ++f)
        if (c.cur[f] != primary_increment(s, f)) {
            cp.src[cp.count] = reinterpret_cast<const double2 *>(c.cur[f]);
            cp.dst[cp.count] = reinterpret_cast<double2 *>(primary_increment(s, f));
            cp.count += 1;
            std::swap(c.cur[f], c.oth[f]);
        }
    if (!cp.count) return HOSC_OK;
    const size_t n = s->g.cs;     // 2 cs doubles = cs pairs
    const unsigned blocks = (unsigned)std::min<size_t>(2048, (n + 255) / 256);
    k_copy4<<<blocks, 256, 0, st>>>(cp, n);
    return launch_check(s, "increment copy");
}

// Decisions after a residual pass, from the reduction block hb (the cavity's
// red[0..55]: ||b/C||^2 at 0..3, dominance at 44..45, FP64 residual sums of the
// red and black halves at 48..51 and 52..55).  Leaves in c.active the groups that
// need another inner solve, with its right-hand-side norms and tolerance.
hosc_status refine_decide(hosc_solver *s, RefCtl &c, const double *hb, double bn2[4], SolveOut &o, double inner_bn2[4],
                          double *inner_rtol)
{
    if (c.outer > 50) return fail(s, HOSC_E_NOCONV, "iterative refinement did not converge in 50 passes");
    const double rtol = s->P.solve_rtol;
    o.dominance[0] = hb[44];
    o.dominance[1] = hb[45];
    if (bn2[0] < 0.0) {
        for (int f = 0; f < 4; ++f) bn2[f] = hb[f];
        for (int f = 0; f < 4; ++f)
            if (!std::isfinite(bn2[f])) return fail(s, HOSC_E_NONFINITE, "non-finite right-hand side");
    }
    double rr[4], target = 0.1;
    for (int f = 0; f < 4; ++f) {
        rr[f] = hb[48 + f] + hb[52 + f];
        inner_bn2[f] = 0.0;
    }
    for (int grp = 0; grp < 2; ++grp) {
        if (!(c.active & (1 << grp))) continue;
        const int f0 = grp == 0 ? 0 : 3, f1 = grp == 0 ? 3 : 4;
        bool conv = true, zero = true;
        for (int f = f0; f < f1; ++f) {
            if (!std::isfinite(rr[f])) return fail(s, HOSC_E_NONFINITE, "non-finite residual in refinement");
            zero = zero && bn2[f] == 0.0;
            o.relres[f] = bn2[f] > 0.0 ? std::sqrt(rr[f] / bn2[f]) : 0.0;
            if (!(bn2[f] == 0.0 || std::sqrt(rr[f]) <= rtol * std::sqrt(bn2[f]))) conv = false;
            inner_bn2[f] = rr[f];
            if (bn2[f] > 0.0 && rr[f] > 0.0) target = std::min(target, rtol * std::sqrt(bn2[f] / rr[f]));
        }
        if (zero) {     // b = 0: the increment is zero
            hosc_status r = zero_group(s, grp);
            if (r) return r;
        }
        if (conv || zero) c.active &= ~(1 << grp);
    }
    // the inner FP32 solve aims at the reduction still needed, but not below 1e-5
    // (its own rounding floor is near 1e-6)
    *inner_rtol = std::max(1e-5, 0.3 * target);
    return HOSC_OK;
}

// After an inner solve: groups whose FP32 solve failed leave the refinement and go
// to the BiCGSTAB fallback; the others' swept systems (momentum fields with a zero
// residual are left out of the sweeps) carry a correction to fold.
hosc_status refine_after_inner(hosc_solver *s, RefCtl &c, int failed, const double inner_bn2[4])
{
    if (failed) {
        for (int grp = 0; grp < 2; ++grp) {
            if (!(failed & (1 << grp))) continue;
            const int f0 = grp == 0 ? 0 : 3, f1 = grp == 0 ? 3 : 4;
            for (int f = f0; f < f1; ++f) {
                HIPCHK(s, hipMemsetAsync(s->fe[f], 0, 2 * s->g.cs * sizeof(float), s->st));
                HIPCHK(s, hipMemsetAsync(s->fr[f], 0, 2 * s->g.cs * sizeof(float), s->st));
            }
        }
        c.to_bicg |= failed;
        c.active &= ~failed;
    }
    c.emask = 0;
    for (int f = 0; f < 4; ++f)
        if ((c.active & (f < 3 ? 1 : 2)) && (f == 3 || inner_bn2[f] != 0.0)) c.emask |= 1 << f;
    c.outer += 1;
    return HOSC_OK;
}

hosc_status refine_loop(hosc_solver *s, RefCtl &c, double bn2[4], SolveOut &o)
{
    const double st = theta_st(s);
    while (c.active) {
        hosc_status r = timed_begin(s);
        if (r) return r;
        const dim3 grd(s->L.grd_sp.x, s->L.grd_sp.y, 2 * s->L.grd_sp.z);
        k_refine_pass<double><<<grd, s->L.blk_sp, 0, s->st>>>(s->g, c.active, c.emask, st, refine_args(s, c),
                                                              s->partR, s->partB);
        r = timed_end(s, 3, refine_bytes(s->g, c.active, c.emask), 1);
        if (r) return r;
        r = launch_check(s, "refinement pass");
        if (r) return r;
        refine_folded(c);
        Reductions()
            .add(s->partR, s->L.nb_sp, 4, 0, s->red + 48, mir(s, s->red + 48))
            .add(s->partB, s->L.nb_sp, 4, 0, s->red + 52, mir(s, s->red + 52))
            .launch(s->st);
        HIPCHK(s, wait_stream(s->st));
        double inner_bn2[4], inner_rtol;
        r = refine_decide(s, c, s->hmir, bn2, o, inner_bn2, &inner_rtol);
        if (r) return r;
        if (!c.active) break;
        int failed = 0;
        s->inner_slot = std::min(c.outer, 1);
        r = run_sor<float>(s, c.active, inner_bn2, o, &failed, sweep_args_fp32(s), inner_rtol, true);
        if (r) return r;
        r = refine_after_inner(s, c, failed, inner_bn2);
        if (r) return r;
    }
    return HOSC_OK;
}

hosc_status solve_refined(hosc_solver *s, int mask, double bn2[4], SolveOut &o, int *to_bicg)
{
    RefCtl c;
    refine_begin(s, c, mask);
    *to_bicg = 0;
    const hosc_status r = refine_loop(s, c, bn2, o);
    const hosc_status r2 = refine_end(s, c, s->st);
    if (r) return r;
    if (r2) return r2;
    *to_bicg = c.to_bicg;
    return HOSC_OK;
}

// Groups solved by SOR (sor_mask) and by BiCGSTAB (bicg_mask) this step.
void solve_masks(const hosc_solver *s, int &sor_mask, int &bicg_mask)
{
    sor_mask = bicg_mask = 0;
    for (int grp = 0; grp < 2; ++grp) {
        const bool use_bicg = s->P.solver == HOSC_SOLVER_BICGSTAB
                              || (s->P.solver == HOSC_SOLVER_AUTO && s->step < s->bicg_until[grp]);
        if (use_bicg) bicg_mask |= 1 << grp;
        else sor_mask |= 1 << grp;
    }
}

// Groups whose SOR solve failed restart from zero under BiCGSTAB (sticky for 50
// steps); then the BiCGSTAB groups are solved.
hosc_status solve_finish(hosc_solver *s, int failed, int bicg_mask, double bn2[4], SolveOut &o)
{
    for (int grp = 0; grp < 2; ++grp)
        if (failed & (1 << grp)) {
            hosc_status r = zero_group(s, grp);     // the SOR iterate may have diverged
            if (r) return r;
            s->bicg_until[grp] = s->step + 50;
            bicg_mask |= 1 << grp;
        }
    hosc_status r = run_bicg<double>(s, bicg_mask, bn2, o, bicg_args<double>(s, s->ms, s->ma, s->ta));
    if (r) return r;
    s->last_bicg[0] = o.bicg[0];
    s->last_bicg[1] = o.bicg[1];
    return HOSC_OK;
}

// Solves the groups in `groups` (1 momentum, 2 energy).
hosc_status solve(hosc_solver *s, SolveOut &o, int groups = 3)
{
    // ||b/C||^2 of the four systems (reduced after the assembly into red[0..3]) are
    // read by the solvers together with their first convergence check
    double bn2[4] = {-1.0, -1.0, -1.0, -1.0};
    int sor_mask, bicg_mask, failed = 0;
    solve_masks(s, sor_mask, bicg_mask);
    sor_mask &= groups;
    bicg_mask &= groups;
    if (sor_mask) {
        hosc_status r = s->fp32 ? solve_refined(s, sor_mask, bn2, o, &failed)
                                : run_sor<double>(s, sor_mask, bn2, o, &failed, sweep_args(s), s->P.solve_rtol);
        if (r) return r;
    }
    return solve_finish(s, failed, bicg_mask, bn2, o);
}

// Assembly of the rows and right-hand sides and its reductions (||b/C||^2 into
// red[0..3], dominance into red[44..45]); with `rows32` the FP32 row copies of the
// precision mode.  Launches only.
hosc_status assemble(hosc_solver *s, bool rows32)
{
    ColourArrays ca;
    ca.ms = s->ms;
    for (int d = 0; d < 3; ++d) {
        ca.ma[d] = s->ma[d];
        ca.mb[d] = s->mb[d];
        ca.ta[d] = s->ta[d];
    }
    ca.tb = s->tb;
    hosc_status r = timed_begin(s);
    if (r) return r;
    const unsigned slab_blocks = s->L.grd_int.x * ((s->L.grd_int.y + 7) / 8) * s->L.grd_int.z * 8;
    k_assemble<<<slab_blocks, s->L.blk_int, 0, s->st>>>(
        s->g, s->ph, s->u, s->v, s->w, s->T, s->eta, s->E[0], s->E[1], s->E[2], s->u2, s->v2, s->w2, s->etap,
        s->Ep[0], s->Ep[1], s->Ep[2], ca, s->partR, s->partB);
    if (s->fp32 && rows32)    // a streaming pass: cheaper than the FP32 stores inside the assembly (register budget)
        k_rows_f32<<<2048, 256, 0, s->st>>>(2 * s->g.cs, s->ms, s->ma[0], s->ma[1], s->ma[2], s->ta[0], s->ta[1],
                                           s->ta[2], s->fms, s->fma[0], s->fma[1], s->fma[2], s->fta[0], s->fta[1],
                                           s->fta[2]);
    r = timed_end(s, 1, assemble_bytes(s->g));
    if (r) return r;
    Reductions()
        .add(s->partR, s->L.nb_int, 4, 0, s->red, mir(s, s->red))
        .add(s->partB, s->L.nb_int, 2, 1, s->red + 44, mir(s, s->red + 44))
        .launch(s->st);
    return launch_check(s, "assemble");
}

// eta, E*, assembly and its reductions; launches only.
hosc_status pre_solve(hosc_solver *s)
{
    hosc_status r = stage_sources(s, true);
    if (r) return r;
    return assemble(s, true);
}

// Pressure iterations of the step (Sec. 2.2): while the trial velocity level n +
// increment has max |div| > div_tol and fewer than p_iters momentum solves were
// made, correct p by -lambda div, re-form the momentum sources of level n with the
// corrected pressure (eta and the rows are unchanged; at the first step level n-1
// follows them) and solve the momentum increments again, warm-started from the
// last ones.  The last solve's divergence and correction are the step's own
// (post_launch / post_finish).
hosc_status pressure_iterations(hosc_solver *s, bool first, SolveOut &so)
{
    for (int it = 1; it < s->P.p_iters; ++it) {
        k_divergence_trial<<<s->L.grd_int, s->L.blk_int, 0, s->st>>>(s->g, s->u, s->v, s->w, s->md[0], s->md[1],
                                                                     s->md[2], s->dbg, s->partR0);
        Reductions().add(s->partR0, s->L.nb_int, 1, 1, s->red + 62, mir(s, s->red + 62)).launch(s->st);
        hosc_status r = launch_check(s, "trial divergence");
        if (r) return r;
        HIPCHK(s, wait_stream(s->st));
        if (!(s->hmir[62] > s->P.div_tol)) break;    // within tolerance (a non-finite value fails later)
        k_pressure_apply<<<s->L.grd_int, s->L.blk_int, 0, s->st>>>(s->g, s->ph, s->dbg, s->p);
        k_p_walls<<<s->L.grd_face, s->L.blk_face, 0, s->st>>>(s->g, s->p);
        so.corrections += 1;
        k_estar<<<s->L.grd_all, s->L.blk_all, 0, s->st>>>(s->g, s->ph, s->u, s->v, s->w, s->T, s->p, s->eta,
                                                           s->E[0], s->E[1], s->E[2]);
        r = launch_check(s, "pressure iteration");
        if (r) return r;
        if (first)
            for (int d = 0; d < 3; ++d)
                HIPCHK(s, hipMemcpyAsync(s->Ep[d], s->E[d], s->g.n3 * sizeof(double), hipMemcpyDeviceToDevice,
                                         s->st));
        r = assemble(s, false);
        if (r) return r;
        SolveOut o2;
        r = solve(s, o2, 1);
        if (r) return r;
        for (int f = 0; f < 3; ++f) so.relres[f] = o2.relres[f];
        so.dominance[0] = o2.dominance[0];
        so.sweeps[0] += o2.sweeps[0];
        so.bicg[0] += o2.bicg[0];
    }
    return HOSC_OK;
}

// Update, theta walls, divergence (with the correction and the pressure walls when
// the correction is not gated), the diagnostics of the new level and the step's
// reductions into red[12..26] and red[56..60], in four launches; launches only.
hosc_status post_launch(hosc_solver *s)
{
    // update: u, v, w into the level n-1 buffers (which become level n+1)
    k_update<<<s->L.grd_int, s->L.blk_int, 0, s->st>>>(s->g, s->u, s->v, s->w, s->u2, s->v2, s->w2, s->T, s->md[0],
                                                       s->md[1], s->md[2], s->td, s->partR);
    // divergence (and the correction when it is not gated) with the theta walls;
    // then the entropy pass, which also leaves eta of level n+1 in the level n-1
    // buffer (level n at the swap), with the pressure walls and the Nusselt rows of
    // level n+1; then every reduction of the step and the Nusselt means (red[12..26],
    // red[56..60])
    const bool gate = s->P.div_tol > 0.0;
    const Geo &g = s->g;
    const int nd = (int)s->L.nb_int, nf = (int)s->L.nb_face, ne = (int)s->L.nb_all;
    k_tail_div_walls<<<nd + nf, 256, 0, s->st>>>(g, s->ph, s->u2, s->v2, s->w2, s->p, gate ? s->dbg : nullptr,
                                                 gate ? 0 : 1, s->partR0, (int)s->L.grd_int.x, (int)s->L.grd_int.y,
                                                 nd, s->T, s->partB, (int)s->L.grd_face.x, (int)s->L.grd_face.y);
    const bool relax = s->P.eta_relax < 1.0;     // level n's viscosity is s->eta until the swap
    const int nfp = gate ? 0 : nf;               // gated: the pressure walls follow the correction (post_finish)
    k_tail_diag<<<ne + nfp + g.N, 256, 0, s->st>>>(g, s->ph, s->wq, s->u2, s->v2, s->w2, s->T, s->etap, s->partB0,
                                                   relax ? s->eta : nullptr, s->P.eta_relax, ne, s->p, nfp,
                                                   (int)s->L.grd_face.x, (int)s->L.grd_face.y, s->nuh, s->nuc,
                                                   s->avh, s->avc, s->mxh);
    Reductions rd;
    rd.add(s->partR, s->L.nb_int, 8, 0, s->red + 12, mir(s, s->red + 12))
        .add(s->partB, s->L.nb_face, 2, 0, s->red + 20, mir(s, s->red + 20))
        .add(s->partR0, s->L.nb_int, 1, 1, s->red + 22, mir(s, s->red + 22))
        .add(s->partB0, s->L.nb_all, 3, 0, s->red + 24, mir(s, s->red + 24));
    k_tail_reduce<<<rd.n + 1, 1024, 0, s->st>>>(rd.r, rd.n, g, s->wq, s->avh, s->avc, s->mxh, s->red + 56,
                                                mir(s, s->red + 56));
    return launch_check(s, "update/divergence/diagnostics");
}

// Number of reduction outputs the step report reads back: red[12 .. 12 + kPost).
constexpr int kPost = 49;

// Diagnostics from the reduction block: Nusselt at red[56..60], entropy sums at
// red[24..26] (hb points at red[base]).
void diag_from(hosc_diag *d, const double *nu, const double *ent)
{
    d->nu_mean_hot = nu[0];
    d->nu_mean_cold = nu[1];
    d->nu_max_hot = nu[2];
    d->nu_max_cold = nu[3];
    d->nu_local_max_hot = nu[4];
    d->e_ht = ent[0];
    d->e_ff = ent[1];
    d->e_total = ent[0] + ent[1];
    d->be_global = d->e_total > 0.0 ? ent[0] / d->e_total : 1.0;
    d->be_mean = ent[2];
}

// Finish the step from hb = red[12 .. 12 + kPost) read back: gated pressure
// correction, pressure walls, level swap, steady residual, diagnostics and the
// step report.
hosc_status post_finish(hosc_solver *s, const double *hb, const SolveOut &so, hosc_step_info *info)
{
    const bool gate = s->P.div_tol > 0.0;
    const double maxdiv = hb[10];
    int corrected = 1;      // ungated: applied (with its walls) by post_launch
    if (gate) {
        corrected = maxdiv > s->P.div_tol;
        if (corrected) {
            k_pressure_apply<<<s->L.grd_int, s->L.blk_int, 0, s->st>>>(s->g, s->ph, s->dbg, s->p);
            k_p_walls<<<s->L.grd_face, s->L.blk_face, 0, s->st>>>(s->g, s->p);
        }
    }
    hosc_status r = launch_check(s, "pressure");
    if (r) return r;
    std::swap(s->u, s->u2);
    std::swap(s->v, s->v2);
    std::swap(s->w, s->w2);
    std::swap(s->eta, s->etap);
    for (int d = 0; d < 3; ++d) std::swap(s->E[d], s->Ep[d]);
    s->step += 1;
    s->eta_ready = true;
    diag_from(&s->diag, hb + 44, hb + 12);
    s->diag_valid = true;
    auto ratio = [](double num, double den) {
        if (den > 0.0) return std::sqrt(num) / std::sqrt(den);
        return num == 0.0 ? 0.0 : HUGE_VAL;
    };
    double res[4];
    res[0] = ratio(hb[0], hb[4]);
    res[1] = ratio(hb[1], hb[5]);
    res[2] = ratio(hb[2], hb[6]);
    res[3] = ratio(hb[3] + hb[8], hb[7] + hb[9]);
    bool finite = std::isfinite(maxdiv);
    for (int f = 0; f < 4; ++f) finite = finite && std::isfinite(res[f]);
    if (info) {
        for (int f = 0; f < 4; ++f) {
            info->res[f] = res[f];
            info->relres[f] = so.relres[f];
        }
        info->maxdiv = maxdiv;
        info->step = s->step;
        info->sweeps[0] = so.sweeps[0];
        info->sweeps[1] = so.sweeps[1];
        info->bicg_iters[0] = so.bicg[0];
        info->bicg_iters[1] = so.bicg[1];
        info->omega[0] = s->om[0];
        info->omega[1] = s->om[1];
        info->dominance[0] = so.dominance[0];
        info->dominance[1] = so.dominance[1];
        info->corrected = corrected + so.corrections;
        info->status = finite ? HOSC_OK : HOSC_E_NONFINITE;
    }
    if (!finite) return fail(s, HOSC_E_NONFINITE, "non-finite steady residual or divergence");
    return HOSC_OK;
}

hosc_status one_step(hosc_solver *s, hosc_step_info *info)
{
    const bool first = s->first;
    hosc_status r = pre_solve(s);
    if (r) return r;
    SolveOut so;
    r = solve(s, so);
    if (r) return r;
    r = pressure_iterations(s, first, so);
    if (r) return r;
    r = post_launch(s);
    if (r) return r;
    HIPCHK(s, wait_stream(s->st));
    return post_finish(s, s->hmir + 12, so, info);
}

// ---------------------------------------------------------------------------
// Fused multi-cavity execution (batches and the server).  The per-cavity phases
// above are reused unchanged; the solver phases, which dominate, run as fused
// launches over every cavity that still iterates: one persistent launch per
// half-sweep, one per refinement pass (both colours), one launch for all the
// reductions and one gather + host copy per convergence check.
// ---------------------------------------------------------------------------
constexpr size_t kCavEntry = 512;     // bytes reserved per cavity for a fused-launch descriptor

struct Fused {
    int cap = 0;                      // cavities the tables hold
    hipStream_t st = nullptr;
    int grid = 1024;                  // persistent workgroups per fused launch (0: one per tile)
    // one contiguous table block, mirrored in pinned host memory: map | cav | jobs | src,
    // then the fixed gather list of the captured post-solve phase
    char *d_tab = nullptr, *h_tab = nullptr;
    size_t off_cav = 0, off_jobs = 0, off_src = 0, tab_bytes = 0, off_src2 = 0;
    // captured pre- and post-solve phases (kind 0 / 1), keyed by the level parity
    // of every cavity; used when the stream is not the null stream
    struct GraphEntry {
        uint64_t sig;
        int kind;
        std::vector<const hosc_solver *> members;   // the cavities of the captured step, in order
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    bool use_graphs = false;
    int64_t graph_launches = 0;
    double *h_gather = nullptr, *h_gather_dev = nullptr;   // mapped host memory the gathers write to
    std::string err;
    bool prof = false;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hosc_perf perf{};
    // side streams (default priority) for the per-cavity phases, and their events
    static constexpr int kSide = 4;
    hipStream_t side[kSide] = {};
    hipEvent_t fork = nullptr, join[kSide] = {};
    TileMap *hmap() { return reinterpret_cast<TileMap *>(h_tab); }
    template <typename T> T *hcav() { return reinterpret_cast<T *>(h_tab + off_cav); }
    ReduceJob *hjobs() { return reinterpret_cast<ReduceJob *>(h_tab + off_jobs); }
    const double **hsrc() { return reinterpret_cast<const double **>(h_tab + off_src); }
    const TileMap *dmap() const { return reinterpret_cast<const TileMap *>(d_tab); }
    template <typename T> const T *dcav() const { return reinterpret_cast<const T *>(d_tab + off_cav); }
    const ReduceJob *djobs() const { return reinterpret_cast<const ReduceJob *>(d_tab + off_jobs); }
    const double *const *dsrc() const { return reinterpret_cast<const double *const *>(d_tab + off_src); }
    const double **hsrc2() { return reinterpret_cast<const double **>(h_tab + off_src2); }
    const double *const *dsrc2() const { return reinterpret_cast<const double *const *>(d_tab + off_src2); }
};

size_t fused_table_bytes(int cap)
{
    return align_up((size_t)cap * sizeof(TileMap)) + align_up((size_t)cap * kCavEntry)
           + align_up((size_t)cap * 4 * sizeof(ReduceJob)) + 2 * align_up((size_t)cap * sizeof(double *));
}
size_t fused_device_bytes(int cap) { return fused_table_bytes(cap); }

hosc_status ffail(Fused &F, hosc_status st, const std::string &msg)
{
    F.err = msg;
    return st;
}
#define FHIPCHK(F, call)                                                                           \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return ffail((F), HOSC_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

// d_dev: device block of fused_device_bytes(cap), 256-byte aligned.
hosc_status fused_init(Fused &F, int cap, char *d_dev, hipStream_t st)
{
    static_assert(sizeof(FusedSweepCav<double, double>) <= kCavEntry, "descriptor too large");
    static_assert(sizeof(FusedSweepCav<float, float>) <= kCavEntry, "descriptor too large");
    static_assert(sizeof(FusedRefineCav<double>) <= kCavEntry, "descriptor too large");
    F.cap = cap;
    F.st = st;
    F.off_cav = align_up((size_t)cap * sizeof(TileMap));
    F.off_jobs = F.off_cav + align_up((size_t)cap * kCavEntry);
    F.off_src = F.off_jobs + align_up((size_t)cap * 4 * sizeof(ReduceJob));
    F.off_src2 = F.off_src + align_up((size_t)cap * sizeof(double *));
    F.tab_bytes = fused_table_bytes(cap);
    F.use_graphs = st != nullptr;
    F.d_tab = d_dev;
    FHIPCHK(F, hipHostMalloc(reinterpret_cast<void **>(&F.h_tab), F.tab_bytes));
    FHIPCHK(F, hipHostMalloc(reinterpret_cast<void **>(&F.h_gather), (size_t)cap * 64 * sizeof(double),
                             hipHostMallocMapped | hipHostMallocCoherent));
    FHIPCHK(F, hipHostGetDevicePointer(reinterpret_cast<void **>(&F.h_gather_dev), F.h_gather, 0));
    std::memset(F.h_tab, 0, F.tab_bytes);
    FHIPCHK(F, hipEventCreate(&F.ev[0]));
    FHIPCHK(F, hipEventCreate(&F.ev[1]));
    if (st != nullptr) {
        FHIPCHK(F, hipEventCreateWithFlags(&F.fork, hipEventDisableTiming));
        for (int q = 0; q < Fused::kSide; ++q) {
            FHIPCHK(F, hipStreamCreateWithFlags(&F.side[q], hipStreamNonBlocking));
            FHIPCHK(F, hipEventCreateWithFlags(&F.join[q], hipEventDisableTiming));
        }
    }
    return HOSC_OK;
}
void fused_free(Fused &F)
{
    for (auto &e : F.graphs) (void)hipGraphExecDestroy(e.exec);
    F.graphs.clear();
    if (F.h_tab) (void)hipHostFree(F.h_tab);
    if (F.h_gather) (void)hipHostFree(F.h_gather);
    for (hipEvent_t &e : F.ev)
        if (e) (void)hipEventDestroy(e);
    for (int q = 0; q < Fused::kSide; ++q) {
        if (F.side[q]) (void)hipStreamDestroy(F.side[q]);
        if (F.join[q]) (void)hipEventDestroy(F.join[q]);
        F.side[q] = nullptr;
        F.join[q] = nullptr;
    }
    if (F.fork) (void)hipEventDestroy(F.fork);
    F.fork = nullptr;
    F.h_tab = nullptr;
    F.h_gather = nullptr;
    F.h_gather_dev = nullptr;
}

void tile_map_of(TileMap &m, dim3 grd, dim3 blk, int &total)
{
    m.tile0 = total;
    m.tiles_x = (int)grd.x;
    m.tiles_y = (int)grd.y;
    m.tiles = m.tiles_x * m.tiles_y * (int)grd.z;
    m.tx = (int)blk.x;
    m.ty = (int)blk.y;
    total += m.tiles;
}
// tiles of the sweep launch (two colour-row entries per thread)
void tile_map_sweep(TileMap &m, const hosc_solver *s, int &total) { tile_map_of(m, s->L.grd_sp, s->L.blk_sp, total); }

int fused_grid(const Fused &F, int total) { return F.grid > 0 ? std::min(F.grid, total) : total; }

// Upload the table block and run the reductions in h_jobs[0..njobs), then gather
// len doubles from each of h_src[0..nsrc) into the mapped h_gather, synchronised.
hosc_status fused_reduce_gather(Fused &F, int njobs, int nsrc, int len)
{
    if (njobs > 0) k_reduce_jobs<<<njobs, 1024, 0, F.st>>>(F.djobs());
    k_gather<<<nsrc, 64, 0, F.st>>>(F.dsrc(), len, F.h_gather_dev);
    FHIPCHK(F, hipGetLastError());
    FHIPCHK(F, wait_stream(F.st));
    return HOSC_OK;
}

void add_job(ReduceJob *jobs, int &n, const double *part, int nb, int nc, int op, double *out)
{
    ReduceJob &j = jobs[n++];
    j.part = part;
    j.nb = nb;
    j.nc = nc;
    j.op = op;
    j.out = out;
    j.out_host = nullptr;
    j.pad = 0;
}

template <typename TM> SweepArgs<TM> cavity_sweep_args(hosc_solver *s);
template <> SweepArgs<double> cavity_sweep_args<double>(hosc_solver *s) { return sweep_args(s); }
template <> SweepArgs<float> cavity_sweep_args<float>(hosc_solver *s) { return sweep_args_fp32(s); }

// Batched red-black SOR over cavities cav[0..n): cavity i solves the groups in
// mask[i] to rtol[i] with exactly the control of run_sor.  A cavity whose control
// reports an error gets it in err[i] and leaves the solve; the others go on.
template <typename TM>
hosc_status fused_sor(Fused &F, hosc_solver *const *cav, int n, const int *mask, double (*bn2)[4], SolveOut *o,
                      int *failed, const double *rtol, bool inner, hosc_status *err)
{
    std::vector<SorCtl> c(n);
    std::vector<SweepArgs<TM>> args(n);
    std::vector<int> act(n);
    bool seed = false;
    for (int i = 0; i < n; ++i) {
        failed[i] = 0;
        if (err[i] || !mask[i]) continue;
        sor_begin(cav[i], c[i], mask[i], rtol[i], inner);
        args[i] = cavity_sweep_args<TM>(cav[i]);
        seed = seed || sor_wants_seed(cav[i], c[i]);
    }
    if (seed) {
        int ns = 0;
        for (int i = 0; i < n; ++i)
            if (!err[i] && mask[i]) {
                F.hsrc()[ns] = cav[i]->red;
                act[ns++] = i;
            }
        FHIPCHK(F, hipMemcpyAsync(F.d_tab, F.h_tab, F.tab_bytes, hipMemcpyHostToDevice, F.st));
        hosc_status r = fused_reduce_gather(F, 0, ns, 48);
        if (r) return r;
        for (int a = 0; a < ns; ++a) {
            const int i = act[a];
            if (sor_wants_seed(cav[i], c[i])) sor_seed(cav[i], c[i], F.h_gather + 48 * a + 44);
            if (bn2[i][0] < 0.0) {
                for (int f = 0; f < 4; ++f) bn2[i][f] = F.h_gather[48 * a + f];
                for (int f = 0; f < 4; ++f)
                    if (!std::isfinite(bn2[i][f])) {
                        err[i] = fail(cav[i], HOSC_E_NONFINITE, "non-finite right-hand side");
                        c[i].active = 0;
                    }
            }
        }
    }
    for (int i = 0; i < n; ++i)
        if (!err[i] && mask[i]) sor_skip(c[i], bn2[i]);
    std::vector<int> order, len(n), upto(n + 1);
    for (;;) {
        int nact = 0, total = 0, nsw = 0, nj = 0;
        double bytes = 0.0;
        // cavities still iterating, the longest batch first: the cavities sweep q
        // reaches are then a prefix of the table, and each launch covers only
        // their tiles (a tile's work does not depend on where it sits in the list)
        order.clear();
        for (int i = 0; i < n; ++i)
            if (!err[i] && c[i].active) order.push_back(i);
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return sor_batch_sweeps(c[a]) > sor_batch_sweeps(c[b]); });
        upto[0] = 0;
        for (const int i : order) {
            hosc_solver *s = cav[i];
            tile_map_sweep(F.hmap()[nact], s, total);
            FusedSweepCav<TM, TM> &cv = F.hcav<FusedSweepCav<TM, TM>>()[nact];
            cv.g = s->g;
            cv.a = args[i];
            cv.omega_m = (TM)s->om[0];
            cv.omega_t = (TM)s->om[1];
            cv.st = (TM)theta_st(s);
            cv.plan_m = (c[i].active & 1) ? c[i].plan[0] : 0;
            cv.plan_t = (c[i].active & 2) ? c[i].plan[1] : 0;
            cv.skip = c[i].skip;
            cv.zs = c[i].zero_start && c[i].batch == 0;
            cv.part[0] = s->partR;
            cv.part[1] = s->partB;
            cv.part0[0] = s->partR0;
            cv.part0[1] = s->partB0;
            const int nb = (int)s->L.nb_sp;
            add_job(F.hjobs(), nj, s->partR, nb, 4, 0, s->red + 4);
            add_job(F.hjobs(), nj, s->partB, nb, 4, 0, s->red + 8);
            add_job(F.hjobs(), nj, s->partR0, nb, 4, 0, s->red + 32);
            add_job(F.hjobs(), nj, s->partB0, nb, 4, 0, s->red + 36);
            F.hsrc()[nact] = s->red;
            const int ns = sor_batch_sweeps(c[i]);
            nsw = std::max(nsw, ns);
            len[nact] = ns;
            upto[nact + 1] = total;
            for (int q = 0; q < ns; ++q) {
                int m;
                unsigned a0, a1;
                sor_sweep_flags(c[i], q, m, a0, a1);
                bytes += 2.0 * sweep_bytes(s->g, m, sizeof(TM));
            }
            act[nact++] = i;
        }
        if (!nact) break;
        FHIPCHK(F, hipMemcpyAsync(F.d_tab, F.h_tab, F.tab_bytes, hipMemcpyHostToDevice, F.st));
        if (F.prof) FHIPCHK(F, hipEventRecord(F.ev[0], F.st));
        int reach = nact;      // cavities whose batch includes sweep q
        for (int q = 0; q < nsw; ++q) {
            while (reach > 0 && len[reach - 1] <= q) --reach;
            const int tq = upto[reach], G = fused_grid(F, tq);
            for (int colour = 0; colour < 2; ++colour)
                k_sweep_fused<TM, TM><<<G, 256, 0, F.st>>>(F.dmap(), F.dcav<FusedSweepCav<TM, TM>>(), reach, tq,
                                                           colour, q);
        }
        if (F.prof) FHIPCHK(F, hipEventRecord(F.ev[1], F.st));
        FHIPCHK(F, hipGetLastError());
        hosc_status r = fused_reduce_gather(F, nj, nact, 48);
        if (r) return r;
        if (F.prof) {
            float ms = 0.0f;
            FHIPCHK(F, hipEventElapsedTime(&ms, F.ev[0], F.ev[1]));
            F.perf.sweep_launches += 2 * nsw;
            F.perf.sweep_ms += ms;
            F.perf.sweep_bytes += bytes;
        }
        for (int a = 0; a < nact; ++a) {
            const int i = order[a];
            r = sor_decide<TM>(cav[i], c[i], F.h_gather + 48 * a, bn2[i], o[i], args[i]);
            if (r) {
                err[i] = r;
                c[i].active = 0;
            }
        }
    }
    for (int i = 0; i < n; ++i) failed[i] = c[i].failed;
    return HOSC_OK;
}

// Batched iterative refinement (precision mode), the control of solve_refined.
hosc_status fused_refined_loop(Fused &F, hosc_solver *const *cav, int n, std::vector<RefCtl> &rc, double (*bn2)[4],
                               SolveOut *o, hosc_status *err)
{
    std::vector<int> act(n), imask(n), ifailed(n);
    std::vector<double> irtol(n);
    std::vector<std::array<double, 4>> ibn2(n);
    for (;;) {
        int nact = 0, total = 0, nj = 0;
        double bytes = 0.0;
        for (int i = 0; i < n; ++i) {
            if (err[i] || !rc[i].active) continue;
            hosc_solver *s = cav[i];
            tile_map_sweep(F.hmap()[nact], s, total);
            FusedRefineCav<double> &cv = F.hcav<FusedRefineCav<double>>()[nact];
            cv.g = s->g;
            cv.a = refine_args(s, rc[i]);
            cv.st = theta_st(s);
            cv.mask = rc[i].active;
            cv.emask = rc[i].emask;
            cv.part[0] = s->partR;
            cv.part[1] = s->partB;
            const int nb = (int)s->L.nb_sp;
            add_job(F.hjobs(), nj, s->partR, nb, 4, 0, s->red + 48);
            add_job(F.hjobs(), nj, s->partB, nb, 4, 0, s->red + 52);
            F.hsrc()[nact] = s->red;
            bytes += refine_bytes(s->g, rc[i].active, rc[i].emask);
            refine_folded(rc[i]);
            act[nact++] = i;
        }
        if (!nact) break;
        FHIPCHK(F, hipMemcpyAsync(F.d_tab, F.h_tab, F.tab_bytes, hipMemcpyHostToDevice, F.st));
        const int G = fused_grid(F, 2 * total);
        if (F.prof) FHIPCHK(F, hipEventRecord(F.ev[0], F.st));
        k_refine_fused<double><<<G, 256, 0, F.st>>>(F.dmap(), F.dcav<FusedRefineCav<double>>(), nact, total);
        if (F.prof) FHIPCHK(F, hipEventRecord(F.ev[1], F.st));
        FHIPCHK(F, hipGetLastError());
        hosc_status r = fused_reduce_gather(F, nj, nact, 56);
        if (r) return r;
        if (F.prof) {
            float ms = 0.0f;
            FHIPCHK(F, hipEventElapsedTime(&ms, F.ev[0], F.ev[1]));
            F.perf.refine_launches += 1;
            F.perf.refine_ms += ms;
            F.perf.refine_bytes += bytes;
        }
        for (int i = 0; i < n; ++i) imask[i] = 0;
        for (int a = 0; a < nact; ++a) {
            const int i = act[a];
            r = refine_decide(cav[i], rc[i], F.h_gather + 56 * a, bn2[i], o[i], ibn2[i].data(), &irtol[i]);
            if (r) {
                err[i] = r;
                rc[i].active = 0;
                continue;
            }
            imask[i] = rc[i].active;
            cav[i]->inner_slot = std::min(rc[i].outer, 1);
        }
        std::vector<double> flat(4 * (size_t)n);
        for (int i = 0; i < n; ++i)
            for (int f = 0; f < 4; ++f) flat[4 * (size_t)i + f] = ibn2[i][f];
        r = fused_sor<float>(F, cav, n, imask.data(), reinterpret_cast<double(*)[4]>(flat.data()), o, ifailed.data(),
                             irtol.data(), true, err);
        if (r) return r;
        for (int i = 0; i < n; ++i) {
            if (!imask[i] || err[i]) continue;
            r = refine_after_inner(cav[i], rc[i], ifailed[i], ibn2[i].data());
            if (r) err[i] = r;
        }
    }
    return HOSC_OK;
}

// Batched iterative refinement (precision mode), the control of solve_refined.
hosc_status fused_refined(Fused &F, hosc_solver *const *cav, int n, const int *mask, double (*bn2)[4], SolveOut *o,
                          int *to_bicg, hosc_status *err)
{
    std::vector<RefCtl> rc(n);
    for (int i = 0; i < n; ++i) refine_begin(cav[i], rc[i], err[i] ? 0 : mask[i]);
    const hosc_status r = fused_refined_loop(F, cav, n, rc, bn2, o, err);
    for (int i = 0; i < n; ++i) {
        const hosc_status r2 = refine_end(cav[i], rc[i], F.st);
        if (r2 && !err[i]) err[i] = r2;
    }
    if (r) return r;
    for (int i = 0; i < n; ++i) to_bicg[i] = rc[i].to_bicg;
    return HOSC_OK;
}

// Level-parity signature of the cavities (bit i: cavity i's level-n buffers are
// swapped); a captured phase bakes the buffer addresses in.
uint64_t parity_sig(hosc_solver *const *cav, int n)
{
    uint64_t sig = 0;
    for (int i = 0; i < n; ++i)
        if (cav[i]->u != cav[i]->u_first) sig |= 1ull << i;
    return sig;
}

// The cavities (in order) a fused step covers: a captured phase replays only for
// the same list (a batch marching to steady state drops cavities as they finish).
std::vector<const hosc_solver *> member_list(hosc_solver *const *cav, int n)
{
    return std::vector<const hosc_solver *>(cav, cav + n);
}

// Replay the captured phase (kind, sig), capturing it first with record() if needed.
template <typename Fn>
hosc_status graph_run(Fused &F, int kind, uint64_t sig, const std::vector<const hosc_solver *> &members, Fn &&record)
{
    for (auto &e : F.graphs)
        if (e.kind == kind && e.sig == sig && e.members == members) {
            FHIPCHK(F, hipGraphLaunch(e.exec, F.st));
            F.graph_launches += 1;
            return HOSC_OK;
        }
    if (F.graphs.size() >= 8) {
        (void)hipGraphExecDestroy(F.graphs.front().exec);
        F.graphs.erase(F.graphs.begin());
    }
    FHIPCHK(F, hipStreamBeginCapture(F.st, hipStreamCaptureModeThreadLocal));
    const hosc_status r = record();
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(F.st, &graph);
    if (r || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (r) return r;
        return ffail(F, HOSC_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return ffail(F, HOSC_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
    F.graphs.push_back({sig, kind, members, exec});
    FHIPCHK(F, hipGraphLaunch(exec, F.st));
    F.graph_launches += 1;
    return HOSC_OK;
}

// Runs fn(i) for each cavity i with use[i] set, with that cavity's launches on side
// stream i mod kSide: the phases of different cavities touch disjoint memory, so
// they run concurrently; F.st then waits for every side stream.  Inside a capture
// the side streams join it through the fork event (one graph branch per stream).
// Without side streams (the null stream) the cavities run in order on their own.
template <typename Fn>
hosc_status fan_out(Fused &F, hosc_solver *const *cav, int n, const int *use, Fn &&fn)
{
    int m = 0;
    for (int i = 0; i < n; ++i) m += use[i] != 0;
    if (!F.side[0] || m < 2) {
        for (int i = 0; i < n; ++i)
            if (use[i]) fn(i);
        return HOSC_OK;
    }
    const int ns = std::min(m, Fused::kSide);
    FHIPCHK(F, hipEventRecord(F.fork, F.st));
    for (int q = 0; q < ns; ++q) FHIPCHK(F, hipStreamWaitEvent(F.side[q], F.fork, 0));
    for (int i = 0, k = 0; i < n; ++i) {
        if (!use[i]) continue;
        hosc_solver *s = cav[i];
        const hipStream_t own = s->st;
        s->st = F.side[k++ % ns];
        fn(i);
        s->st = own;
    }
    for (int q = 0; q < ns; ++q) {
        FHIPCHK(F, hipEventRecord(F.join[q], F.side[q]));
        FHIPCHK(F, hipStreamWaitEvent(F.st, F.join[q], 0));
    }
    return HOSC_OK;
}

// One step of every cavity in cav[0..n) (all of one precision).  Per-cavity
// failures are returned in err[i] (and make that solver sticky, as hosc_step
// does); the return value reports failures of the fused machinery itself.
hosc_status fused_step(Fused &F, hosc_solver *const *cav, int n, hosc_step_info *info, hosc_status *err)
{
    std::vector<SolveOut> o(n);
    std::vector<double> bn2(4 * (size_t)n, -1.0);
    std::vector<int> sor(n), bic(n), failed(n), act(n), first(n);
    for (int i = 0; i < n; ++i) first[i] = cav[i]->first;
    std::vector<double> rtol(n);
    // the pre- and post-solve phases of steady-going batches run as captured graphs
    bool graphed = F.use_graphs && n <= 64;
    for (int i = 0; i < n; ++i) {
        const hosc_solver *s = cav[i];
        graphed = graphed && s->has_state && !s->sticky && !s->first && !s->prof;
    }
    const uint64_t sig = graphed ? parity_sig(cav, n) : 0;
    const std::vector<const hosc_solver *> members = graphed ? member_list(cav, n) : std::vector<const hosc_solver *>();
    std::vector<int> all(n, 1);
    if (graphed) {
        hosc_status r = graph_run(F, 0, sig, members, [&]() {
            hosc_status first_err = HOSC_OK;
            std::string msg;
            hosc_status fr = fan_out(F, cav, n, all.data(), [&](int i) {
                hosc_status q = pre_solve(cav[i]);
                if (q && !first_err) {
                    first_err = q;
                    msg = "cavity " + std::to_string(i) + ": " + cav[i]->err;
                }
            });
            if (fr) return fr;
            return first_err ? ffail(F, first_err, msg) : HOSC_OK;
        });
        if (r) return r;
    }
    std::vector<int> go(n, 0);
    for (int i = 0; i < n; ++i) {
        err[i] = HOSC_OK;
        hosc_solver *s = cav[i];
        if (!s->has_state) err[i] = fail(s, HOSC_E_STATE, "no state set");
        else if (s->sticky) err[i] = fail(s, HOSC_E_STATE, "solver is in an error state; set a new state");
        else go[i] = !graphed;
    }
    {
        hosc_status r = fan_out(F, cav, n, go.data(), [&](int i) { err[i] = pre_solve(cav[i]); });
        if (r) return r;
    }
    for (int i = 0; i < n; ++i) {
        hosc_solver *s = cav[i];
        solve_masks(s, sor[i], bic[i]);
        rtol[i] = s->P.solve_rtol;
        if (err[i]) sor[i] = bic[i] = 0;
    }
    double(*b4)[4] = reinterpret_cast<double(*)[4]>(bn2.data());
    const bool fp32 = n > 0 && cav[0]->fp32;
    hosc_status r = fp32 ? fused_refined(F, cav, n, sor.data(), b4, o.data(), failed.data(), err)
                         : fused_sor<double>(F, cav, n, sor.data(), b4, o.data(), failed.data(), rtol.data(), false, err);
    if (r) return r;
    int nact = 0;
    for (int i = 0; i < n; ++i) {
        if (err[i]) continue;
        err[i] = solve_finish(cav[i], failed[i], bic[i], b4[i], o[i]);
        // pressure iterations with the single-cavity solves (the same control as the
        // fused ones, so results stay those of the cavity alone)
        if (!err[i]) err[i] = pressure_iterations(cav[i], first[i], o[i]);
        if (err[i]) continue;
        act[nact++] = i;
    }
    if (graphed && nact == n) {
        // fixed gather list of the captured phase: red[12..22] of every cavity in order
        bool fresh = false;
        for (int i = 0; i < n; ++i)
            if (F.hsrc2()[i] != cav[i]->red + 12) {
                F.hsrc2()[i] = cav[i]->red + 12;
                fresh = true;
            }
        if (fresh)
            FHIPCHK(F, hipMemcpyAsync(F.d_tab + F.off_src2, F.h_tab + F.off_src2, (size_t)n * sizeof(double *),
                                      hipMemcpyHostToDevice, F.st));
        r = graph_run(F, 1, sig, members, [&]() {
            hosc_status first_err = HOSC_OK;
            std::string msg;
            hosc_status fr = fan_out(F, cav, n, all.data(), [&](int i) {
                hosc_status q = post_launch(cav[i]);
                if (q && !first_err) {
                    first_err = q;
                    msg = "cavity " + std::to_string(i) + ": " + cav[i]->err;
                }
            });
            if (fr) return fr;
            if (first_err) return ffail(F, first_err, msg);
            k_gather<<<n, 64, 0, F.st>>>(F.dsrc2(), kPost, F.h_gather_dev);
            return HOSC_OK;
        });
        if (r) return r;
        FHIPCHK(F, wait_stream(F.st));
    } else if (nact) {
        std::vector<int> post(n, 0);
        for (int a = 0; a < nact; ++a) post[act[a]] = 1;
        r = fan_out(F, cav, n, post.data(), [&](int i) { err[i] = post_launch(cav[i]); });
        if (r) return r;
        int ng = 0;
        for (int a = 0; a < nact; ++a) {
            const int i = act[a];
            if (!err[i]) {
                F.hsrc()[ng] = cav[i]->red + 12;
                act[ng++] = i;
            }
        }
        nact = ng;
        if (nact) {
            FHIPCHK(F, hipMemcpyAsync(F.d_tab + F.off_src, F.h_tab + F.off_src, (size_t)nact * sizeof(double *),
                                      hipMemcpyHostToDevice, F.st));
            r = fused_reduce_gather(F, 0, nact, kPost);
            if (r) return r;
        }
    }
    for (int a = 0; a < nact; ++a) {
        const int i = act[a];
        err[i] = post_finish(cav[i], F.h_gather + kPost * a, o[i], info ? &info[i] : nullptr);
    }
    for (int i = 0; i < n; ++i)
        if (err[i]) {
            if (err[i] == HOSC_E_NOCONV || err[i] == HOSC_E_NONFINITE) cav[i]->sticky = err[i];
            if (info) info[i].status = err[i];
        }
    return HOSC_OK;
}

// Time a few fused half-sweep pairs at each candidate schedule and keep the
// fastest.  Sweeps change the increments, so this runs only on fresh states and
// zeroes the increments afterwards.
template <typename TM>
hosc_status fused_tune(Fused &F, hosc_solver *const *cav, int n, int *best_grid)
{
    int total = 0;
    for (int i = 0; i < n; ++i) {
        hosc_solver *s = cav[i];
        tile_map_sweep(F.hmap()[i], s, total);
        FusedSweepCav<TM, TM> &cv = F.hcav<FusedSweepCav<TM, TM>>()[i];
        cv.g = s->g;
        cv.a = cavity_sweep_args<TM>(s);
        cv.omega_m = cv.omega_t = (TM)1;
        cv.st = (TM)theta_st(s);
        cv.plan_m = cv.plan_t = 1;
        cv.skip = 0;
        cv.zs = 0;
        cv.part[0] = s->partR;
        cv.part[1] = s->partB;
        cv.part0[0] = s->partR0;
        cv.part0[1] = s->partB0;
    }
    FHIPCHK(F, hipMemcpyAsync(F.d_tab, F.h_tab, F.tab_bytes, hipMemcpyHostToDevice, F.st));
    const int cand[] = {256, 512, 1024, 2048, 4096, 0};
    double best = HUGE_VAL;
    int bg = F.grid;
    for (int g : cand) {
        const int G = g > 0 ? std::min(g, total) : total;
        float ms = 0.0f;
        for (int rep = 0; rep < 4; ++rep) {
            if (rep == 1) FHIPCHK(F, hipEventRecord(F.ev[0], F.st));
            for (int colour = 0; colour < 2; ++colour)
                k_sweep_fused<TM, TM><<<G, 256, 0, F.st>>>(F.dmap(), F.dcav<FusedSweepCav<TM, TM>>(), n, total,
                                                           colour, 0);
        }
        FHIPCHK(F, hipEventRecord(F.ev[1], F.st));
        FHIPCHK(F, hipGetLastError());
        FHIPCHK(F, hipEventSynchronize(F.ev[1]));
        FHIPCHK(F, hipEventElapsedTime(&ms, F.ev[0], F.ev[1]));
        if (ms < best) {
            best = ms;
            bg = g;
        }
    }
    F.grid = bg;
    *best_grid = bg;
    for (int i = 0; i < n; ++i) {
        hosc_status r = zero_colour_increments(cav[i]);
        if (r) return ffail(F, r, cav[i]->err);
    }
    return HOSC_OK;
}

}  // namespace

struct hosc_batch {
    std::vector<hosc_solver *> cav;
    Fused F;
    hipStream_t st = nullptr;
    bool fp32 = false;
    std::string err;
};

struct hosc_server {
    struct Req {
        uint64_t id;
        hosc_request rq;
        size_t bytes;
    };
    struct Res {
        Req q;
        hosc_solver *s;
        size_t off;
        double t_admit;
        int64_t steps;
        double res;
    };
    char *arena = nullptr;
    size_t budget = 0, in_use = 0, peak = 0;
    std::map<size_t, size_t> free_;     // offset -> bytes, coalesced
    int max_resident = 0;
    char *d_fused = nullptr;
    Fused F;
    hipStream_t st = nullptr;
    std::deque<Req> queue;
    std::vector<Res> res;
    std::deque<hosc_result> done;
    uint64_t next_id = 1;
    int64_t server_steps = 0, cavity_steps = 0, completed = 0;
    double busy_s = 0.0;
    std::chrono::steady_clock::time_point t0;
    std::string err;
    double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace {

hosc_status sfail(hosc_server *v, hosc_status st, const std::string &msg)
{
    if (v) v->err = msg;
    else g_create_error = msg;
    return st;
}

// First fit in the arena (sizes 256-byte multiples); SIZE_MAX when nothing fits.
size_t arena_alloc(hosc_server *v, size_t bytes)
{
    for (auto it = v->free_.begin(); it != v->free_.end(); ++it)
        if (it->second >= bytes) {
            const size_t off = it->first, rest = it->second - bytes;
            v->free_.erase(it);
            if (rest) v->free_[off + bytes] = rest;
            v->in_use += bytes;
            v->peak = std::max(v->peak, v->in_use);
            return off;
        }
    return SIZE_MAX;
}
void arena_free(hosc_server *v, size_t off, size_t bytes)
{
    v->in_use -= bytes;
    auto it = v->free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != v->free_.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        v->free_.erase(nx);
    }
    if (it != v->free_.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            v->free_.erase(it);
        }
    }
}

// Retire resident cavity k (swap-removed) with status st.
void server_retire(hosc_server *v, size_t k, hosc_status st, bool steady)
{
    hosc_server::Res &r = v->res[k];
    hosc_result out{};
    out.id = r.q.id;
    out.status = st;
    out.steady = steady ? 1 : 0;
    out.steps = r.steps;
    out.res = r.res;
    out.t_arrival = r.q.rq.t_arrival;
    out.t_admit = r.t_admit;
    if (st == HOSC_OK) {
        const hosc_status d = hosc_diagnostics(r.s, &out.diag, nullptr, nullptr, nullptr, nullptr);
        if (d) out.status = d;
    }
    out.t_done = v->now();
    v->done.push_back(out);
    hosc_destroy(r.s);
    arena_free(v, r.off, r.q.bytes);
    v->completed += 1;
    v->res[k] = v->res.back();
    v->res.pop_back();
}

}  // namespace

namespace {

hosc_status bfail(hosc_batch *b, hosc_status st, const std::string &msg)
{
    if (b) b->err = msg;
    else g_create_error = msg;
    return st;
}

size_t batch_layout(const hosc_params *p, int count, std::vector<size_t> *offsets)
{
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        Geo g = make_geo(p[i].N);
        Launch L = make_launch(g);
        if (offsets) offsets->push_back(off);
        off += align_up(make_layout(g, L, p[i].solver, p[i].precision).total_bytes);
    }
    if (offsets) offsets->push_back(off);
    return off + fused_device_bytes(count);
}

// Mean kernel time of `reps` launches of `launch` on `stream`, after one untimed
// warm-up launch (HIP events; both events are released on every path).
template <typename F>
hipError_t time_launches(hipStream_t stream, int reps, F launch, double *ms_per_launch)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        launch();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e0, stream);
    for (int q = 0; q < reps && e == hipSuccess; ++q) launch();
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(e1, stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e == hipSuccess) *ms_per_launch = ms / reps;
    return e;
}

}  // namespace

extern "C" {

hosc_status hosc_params_default(hosc_params *p)
{
    if (!p) return HOSC_E_ARG;
    std::memset(p, 0, sizeof(*p));
    p->N = 17;
    p->precision = HOSC_FP64;
    p->Ra = 1e3;
    p->Pr = 1.0;
    p->n_pl = 1.0;
    p->dt = 1e-4;
    p->theta_hot = 1.0;
    p->theta_cold = 0.0;
    p->theta_ref = 0.5;
    p->lambda = 0.0;
    p->div_tol = 0.0;
    p->solve_rtol = 1e-10;
    p->solve_maxit = 4000;
    p->check_every = 0;
    p->solver = HOSC_SOLVER_AUTO;
    p->p_iters = 1;
    p->omega = 0.0;
    p->i2_floor = 1e-8;
    p->phi = 1e-4;
    p->eta_relax = 1.0;
    return HOSC_OK;
}

hosc_status hosc_workspace_bytes(const hosc_params *p, size_t *bytes)
{
    const char *e = check_params(p);
    if (e) return fail(nullptr, HOSC_E_ARG, e);
    if (!bytes) return fail(nullptr, HOSC_E_ARG, "bytes is NULL");
    Geo g = make_geo(p->N);
    Launch L = make_launch(g);
    *bytes = make_layout(g, L, p->solver, p->precision).total_bytes;
    return HOSC_OK;
}

hosc_status hosc_create(const hosc_params *p, void *d_ws, size_t ws_bytes, hipStream_t stream, hosc_solver **out)
{
    if (!out) return fail(nullptr, HOSC_E_ARG, "out is NULL");
    *out = nullptr;
    const char *e = check_params(p);
    if (e) return fail(nullptr, HOSC_E_ARG, e);
    if (!d_ws) return fail(nullptr, HOSC_E_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return fail(nullptr, HOSC_E_ARG, "workspace must be 256-byte aligned");
    hosc_solver *s = new (std::nothrow) hosc_solver();
    if (!s) return fail(nullptr, HOSC_E_NOMEM, "host allocation failed");
    s->P = *p;
    s->g = make_geo(p->N);
    s->L = make_launch(s->g);
    s->Y = make_layout(s->g, s->L, p->solver, p->precision);
    if (ws_bytes < s->Y.total_bytes) {
        delete s;
        return fail(nullptr, HOSC_E_NOMEM, "workspace smaller than hosc_workspace_bytes()");
    }
    const double h = s->g.h;
    s->ph.Ra = p->Ra;
    s->ph.Pr = p->Pr;
    s->ph.dt = p->dt;
    s->ph.theta_hot = p->theta_hot;
    s->ph.theta_cold = p->theta_cold;
    s->ph.theta_ref = p->theta_ref;
    s->ph.i2_floor = p->i2_floor;
    s->ph.ex = 0.5 * (p->n_pl - 1.0);
    s->ph.lambda = p->lambda > 0.0 ? p->lambda : h * h / (3.0 * p->dt);
    s->ph.phi = p->phi;
    s->st = stream;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(nullptr, HOSC_E_DEVICE, "hipGetDevice failed");
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&s->hbuf), 64 * sizeof(double)) != hipSuccess) {
        delete s;
        return fail(nullptr, HOSC_E_DEVICE, "hipHostMalloc of the staging buffer failed");
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&s->hmir), kRed * sizeof(double),
                      hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess
        || hipHostGetDevicePointer(reinterpret_cast<void **>(&s->hmir_dev), s->hmir, 0) != hipSuccess) {
        if (s->hmir) (void)hipHostFree(s->hmir);
        (void)hipHostFree(s->hbuf);
        delete s;
        return fail(nullptr, HOSC_E_DEVICE, "hipHostMalloc of the mapped reduction mirror failed");
    }
    std::memset(s->hmir, 0, kRed * sizeof(double));
    carve(s, static_cast<char *>(d_ws));
    std::vector<double> wq = simpson(p->N);
    hipError_t he = hipMemcpy(s->wq, wq.data(), wq.size() * sizeof(double), hipMemcpyHostToDevice);
    if (he != hipSuccess) {
        (void)hipHostFree(s->hbuf);
        (void)hipHostFree(s->hmir);
        delete s;
        return fail(nullptr, HOSC_E_DEVICE, std::string("copy of quadrature weights: ") + hipGetErrorString(he));
    }
    *out = s;
    return HOSC_OK;
}

hosc_status hosc_destroy(hosc_solver *s)
{
    if (!s) return HOSC_OK;
    (void)hipStreamSynchronize(s->st);
    for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
    if (s->hbuf) (void)hipHostFree(s->hbuf);
    if (s->hmir) (void)hipHostFree(s->hmir);
    delete s;
    return HOSC_OK;
}

hosc_status hosc_set_state(hosc_solver *s, const double *u, const double *v, const double *w, const double *theta,
                           const double *p, int32_t apply_bc)
{
    if (!s) return HOSC_E_ARG;
    const size_t b = s->g.n3 * sizeof(double);
    double *dst[5] = {s->u, s->v, s->w, s->T, s->p};
    const double *src[5] = {u, v, w, theta, p};
    for (int f = 0; f < 5; ++f) {
        if (src[f]) HIPCHK(s, hipMemcpyAsync(dst[f], src[f], b, hipMemcpyHostToDevice, s->st));
        else HIPCHK(s, hipMemsetAsync(dst[f], 0, b, s->st));
    }
    if (apply_bc) {
        hosc_status r = impose_bc(s);
        if (r) return r;
    }
    return reset_state(s);
}

hosc_status hosc_init_fields(hosc_solver *s, uint64_t seed, double noise_amp)
{
    if (!s) return HOSC_E_ARG;
    if (!std::isfinite(noise_amp)) return fail(s, HOSC_E_ARG, "noise_amp must be finite");
    const int N = s->g.N, M = N - 2;
    std::vector<double> T(s->g.n3);
    const double th = s->P.theta_hot, tc = s->P.theta_cold;
    uint64_t draw = 0;
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                const double x = (double)i / (N - 1);
                double t = th + (tc - th) * x;
                const bool interior = i > 0 && j > 0 && k > 0 && i < N - 1 && j < N - 1 && k < N - 1;
                if (interior && noise_amp != 0.0 && M > 0) {
                    const double U = (double)(splitmix64(seed, draw) >> 11) * 0x1.0p-53;
                    t += noise_amp * (2.0 * U - 1.0);
                }
                if (interior) ++draw;
                T[(size_t)i + (size_t)N * ((size_t)j + (size_t)N * k)] = t;
            }
    return hosc_set_state(s, nullptr, nullptr, nullptr, T.data(), nullptr, 1);
}

hosc_status hosc_get_state(hosc_solver *s, double *u, double *v, double *w, double *theta, double *p)
{
    if (!s) return HOSC_E_ARG;
    if (!s->has_state) return fail(s, HOSC_E_STATE, "no state set");
    const size_t b = s->g.n3 * sizeof(double);
    double *dst[5] = {u, v, w, theta, p};
    const double *src[5] = {s->u, s->v, s->w, s->T, s->p};
    for (int f = 0; f < 5; ++f)
        if (dst[f]) HIPCHK(s, hipMemcpyAsync(dst[f], src[f], b, hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    return HOSC_OK;
}

hosc_status hosc_step(hosc_solver *s, int32_t nsteps, hosc_step_info *info)
{
    if (!s) return HOSC_E_ARG;
    if (nsteps < 0) return fail(s, HOSC_E_ARG, "nsteps must be >= 0");
    if (!s->has_state) return fail(s, HOSC_E_STATE, "no state set");
    if (s->sticky) return fail(s, HOSC_E_STATE, "solver is in an error state; set a new state");
    for (int q = 0; q < nsteps; ++q) {
        hosc_status r = one_step(s, info);
        if (r) {
            if (r == HOSC_E_NOCONV || r == HOSC_E_NONFINITE) s->sticky = r;
            if (info) info->status = r;
            return r;
        }
    }
    return HOSC_OK;
}

hosc_status hosc_run_to_steady(hosc_solver *s, double res_tol, int64_t max_steps, hosc_step_info *info)
{
    if (!s) return HOSC_E_ARG;
    if (!(res_tol > 0.0)) return fail(s, HOSC_E_ARG, "res_tol must be > 0");
    if (max_steps < 0) return fail(s, HOSC_E_ARG, "max_steps must be >= 0");
    if (!s->has_state) return fail(s, HOSC_E_STATE, "no state set");
    if (s->sticky) return fail(s, HOSC_E_STATE, "solver is in an error state; set a new state");
    hosc_step_info local;
    hosc_step_info *ip = info ? info : &local;
    for (int64_t q = 0; q < max_steps; ++q) {
        hosc_status r = hosc_step(s, 1, ip);
        if (r) return r;
        const double m = std::max(std::max(ip->res[0], ip->res[1]), std::max(ip->res[2], ip->res[3]));
        if (m < res_tol) return HOSC_OK;
    }
    return HOSC_OK;
}

hosc_status hosc_diagnostics(hosc_solver *s, hosc_diag *d, double *nuavg_hot, double *nuavg_cold, double *nu_hot,
                             double *nu_cold)
{
    if (!s || !d) return HOSC_E_ARG;
    if (!s->has_state) return fail(s, HOSC_E_STATE, "no state set");
    const Geo &g = s->g;
    const size_t nb = (size_t)g.N * sizeof(double), n2 = (size_t)g.N * g.N * sizeof(double);
    if (s->diag_valid) {    // computed at the end of the step that produced this state
        *d = s->diag;
        if (nuavg_hot) HIPCHK(s, hipMemcpyAsync(nuavg_hot, s->avh, nb, hipMemcpyDeviceToHost, s->st));
        if (nuavg_cold) HIPCHK(s, hipMemcpyAsync(nuavg_cold, s->avc, nb, hipMemcpyDeviceToHost, s->st));
        if (nu_hot) HIPCHK(s, hipMemcpyAsync(nu_hot, s->nuh, n2, hipMemcpyDeviceToHost, s->st));
        if (nu_cold) HIPCHK(s, hipMemcpyAsync(nu_cold, s->nuc, n2, hipMemcpyDeviceToHost, s->st));
        if (nuavg_hot || nuavg_cold || nu_hot || nu_cold) HIPCHK(s, hipStreamSynchronize(s->st));
        return HOSC_OK;
    }
    k_nu_rows<<<g.N, 256, 0, s->st>>>(g, s->wq, s->T, s->nuh, s->nuc, s->avh, s->avc, s->mxh);
    k_nu_final<<<1, 1024, 0, s->st>>>(g, s->wq, s->avh, s->avc, s->mxh, s->nuout);
    k_entropy<<<s->L.grd_all, s->L.blk_all, 0, s->st>>>(g, s->ph, s->wq, s->u, s->v, s->w, s->T, nullptr, nullptr,
                                                         nullptr, s->partR);
    k_reduce<<<1, 1024, 0, s->st>>>(s->partR, (int)s->L.nb_all, 3, 0, s->red + 24);
    hosc_status r = launch_check(s, "diagnostics");
    if (r) return r;
    HIPCHK(s, hipMemcpyAsync(s->hbuf, s->nuout, 5 * sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipMemcpyAsync(s->hbuf + 8, s->red + 24, 3 * sizeof(double), hipMemcpyDeviceToHost, s->st));
    if (nuavg_hot) HIPCHK(s, hipMemcpyAsync(nuavg_hot, s->avh, nb, hipMemcpyDeviceToHost, s->st));
    if (nuavg_cold) HIPCHK(s, hipMemcpyAsync(nuavg_cold, s->avc, nb, hipMemcpyDeviceToHost, s->st));
    if (nu_hot) HIPCHK(s, hipMemcpyAsync(nu_hot, s->nuh, n2, hipMemcpyDeviceToHost, s->st));
    if (nu_cold) HIPCHK(s, hipMemcpyAsync(nu_cold, s->nuc, n2, hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    diag_from(d, s->hbuf, s->hbuf + 8);
    s->diag = *d;
    s->diag_valid = true;
    return HOSC_OK;
}

hosc_status hosc_entropy_fields(hosc_solver *s, double *e_local, double *be_local)
{
    if (!s) return HOSC_E_ARG;
    if (!s->has_state) return fail(s, HOSC_E_STATE, "no state set");
    // each field goes through the scratch array and is copied out before the next
    k_entropy<<<s->L.grd_all, s->L.blk_all, 0, s->st>>>(s->g, s->ph, s->wq, s->u, s->v, s->w, s->T, s->dbg,
                                                         nullptr, nullptr, s->partR);
    hosc_status r = launch_check(s, "entropy");
    if (r) return r;
    const size_t b = s->g.n3 * sizeof(double);
    if (e_local) HIPCHK(s, hipMemcpyAsync(e_local, s->dbg, b, hipMemcpyDeviceToHost, s->st));
    if (be_local) {
        k_entropy<<<s->L.grd_all, s->L.blk_all, 0, s->st>>>(s->g, s->ph, s->wq, s->u, s->v, s->w, s->T, nullptr,
                                                             s->dbg, nullptr, s->partR);
        r = launch_check(s, "entropy");
        if (r) return r;
        HIPCHK(s, hipMemcpyAsync(be_local, s->dbg, b, hipMemcpyDeviceToHost, s->st));
    }
    HIPCHK(s, hipStreamSynchronize(s->st));
    return HOSC_OK;
}

hosc_status hosc_probe(hosc_solver *s, const double *xyz, int32_t n, double *out)
{
    if (!s) return HOSC_E_ARG;
    if (!xyz || !out) return fail(s, HOSC_E_ARG, "xyz and out are required");
    const size_t cap = std::min<size_t>(4096, s->g.n3 / 8);
    if (n < 1 || (size_t)n > cap)
        return fail(s, HOSC_E_ARG, "n must be in [1, min(4096, N^3/8)] (" + std::to_string(cap) + " here)");
    for (int i = 0; i < 3 * n; ++i)
        if (!(xyz[i] >= 0.0 && xyz[i] <= 1.0)) return fail(s, HOSC_E_ARG, "probe coordinates must lie in [0, 1]");
    if (!s->has_state) return fail(s, HOSC_E_STATE, "no state set");
    // points and results staged in the scratch array (3n + 5n <= N^3 doubles)
    double *dx = s->dbg, *dout = s->dbg + 3 * (size_t)n;
    HIPCHK(s, hipMemcpyAsync(dx, xyz, 3 * (size_t)n * sizeof(double), hipMemcpyHostToDevice, s->st));
    k_probe<<<(n + 255) / 256, 256, 0, s->st>>>(s->g, s->u, s->v, s->w, s->T, s->p, dx, n, dout);
    hosc_status r = launch_check(s, "probe");
    if (r) return r;
    HIPCHK(s, hipMemcpyAsync(out, dout, 5 * (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    return HOSC_OK;
}

hosc_status hosc_debug_assemble(hosc_solver *s, double *eta, double *estar, double *b, double *Bmom, double *Btheta)
{
    if (!s) return HOSC_E_ARG;
    if (!s->has_state) return fail(s, HOSC_E_STATE, "no state set");
    hosc_status r = stage_sources(s, false);
    if (r) return r;
    const size_t nb = s->g.n3 * sizeof(double);
    if (eta) HIPCHK(s, hipMemcpyAsync(eta, s->eta, nb, hipMemcpyDeviceToHost, s->st));
    for (int d = 0; d < 3; ++d)
        if (estar) HIPCHK(s, hipMemcpyAsync(estar + d * s->g.n3, s->E[d], nb, hipMemcpyDeviceToHost, s->st));
    for (int what = 0; what < 18; ++what) {
        double *dst = nullptr;
        if (what < 7) dst = Bmom ? Bmom + (size_t)what * s->g.n3 : nullptr;
        else if (what < 14) dst = Btheta ? Btheta + (size_t)(what - 7) * s->g.n3 : nullptr;
        else dst = b ? b + (size_t)(what - 14) * s->g.n3 : nullptr;
        if (!dst) continue;
        HIPCHK(s, hipMemsetAsync(s->dbg, 0, nb, s->st));
        k_assemble_debug<<<s->L.grd_int, s->L.blk_int, 0, s->st>>>(
            s->g, s->ph, s->u, s->v, s->w, s->T, s->eta, s->E[0], s->E[1], s->E[2], s->u2, s->v2, s->w2, s->etap,
            s->Ep[0], s->Ep[1], s->Ep[2], what, s->dbg);
        r = launch_check(s, "assemble_debug");
        if (r) return r;
        HIPCHK(s, hipMemcpyAsync(dst, s->dbg, nb, hipMemcpyDeviceToHost, s->st));
        HIPCHK(s, hipStreamSynchronize(s->st));
    }
    HIPCHK(s, hipStreamSynchronize(s->st));
    return HOSC_OK;
}

hosc_status hosc_transport_step(hosc_solver *s, const double *L, const double *G, const double *H, const double *I,
                                const double *E, const double *Lp, const double *Gp, const double *Hp,
                                const double *Ip, const double *Ep, const double *chi, double *chi_new,
                                hosc_step_info *info)
{
    if (!s) return HOSC_E_ARG;
    if (!L || !G || !H || !I || !Lp || !Gp || !Hp || !Ip || !chi || !chi_new)
        return fail(s, HOSC_E_ARG, "L, G, H, I at both levels, chi and chi_new are required");
    if (!E != !Ep) return fail(s, HOSC_E_ARG, "E and Ep must both be given or both be NULL");
    // the workspace's natural arrays hold the coefficients: the solver's state is gone
    s->has_state = false;
    s->sticky = HOSC_OK;
    const size_t nb = s->g.n3 * sizeof(double);
    double *dL = s->eta, *dG = s->u, *dH = s->v, *dI = s->w, *dE = s->E[0];
    double *dLp = s->etap, *dGp = s->u2, *dHp = s->v2, *dIp = s->w2, *dEp = s->Ep[0];
    double *dchi = s->T, *dnew = s->p;
    const double *src[12] = {L, G, H, I, E, Lp, Gp, Hp, Ip, Ep, chi, chi_new};
    double *dst[12] = {dL, dG, dH, dI, dE, dLp, dGp, dHp, dIp, dEp, dchi, dnew};
    for (int q = 0; q < 12; ++q)
        if (src[q]) HIPCHK(s, hipMemcpyAsync(dst[q], src[q], nb, hipMemcpyHostToDevice, s->st));
    // a fresh solve: zero increments, no inherited sweep plan or relaxation
    hosc_status r = zero_colour_increments(s);
    if (r) return r;
    s->step = 0;
    s->first = true;
    s->last_sweeps[0] = s->last_sweeps[1] = 0;
    for (auto &h : s->inner_sweeps) h[0] = h[1] = 0;
    s->last_bicg[0] = s->last_bicg[1] = 0;
    s->bicg_until[0] = s->bicg_until[1] = -1;
    s->om[0] = s->om[1] = s->P.omega > 0.0 ? s->P.omega : 1.0;
    s->seeded_at = -1;
    s->eta_ready = false;
    s->diag_valid = false;
    ColourArrays ca;
    ca.ms = s->ms;
    for (int d = 0; d < 3; ++d) {
        ca.ma[d] = s->ma[d];
        ca.mb[d] = s->mb[d];
        ca.ta[d] = s->ta[d];
    }
    ca.tb = s->tb;
    k_assemble_transport<<<s->L.grd_int, s->L.blk_int, 0, s->st>>>(s->g, s->P.dt, dL, dG, dH, dI, E ? dE : nullptr,
                                                                   dLp, dGp, dHp, dIp, E ? dEp : nullptr, dchi, dnew,
                                                                   ca, s->partR, s->partB);
    if (s->fp32)
        k_rows_f32<<<2048, 256, 0, s->st>>>(2 * s->g.cs, s->ms, s->ma[0], s->ma[1], s->ma[2], s->ta[0], s->ta[1],
                                           s->ta[2], s->fms, s->fma[0], s->fma[1], s->fma[2], s->fta[0], s->fta[1],
                                           s->fta[2]);
    Reductions()
        .add(s->partR, s->L.nb_int, 4, 0, s->red, mir(s, s->red))
        .add(s->partB, s->L.nb_int, 2, 1, s->red + 44, mir(s, s->red + 44))
        .launch(s->st);
    r = launch_check(s, "transport assembly");
    if (r) return r;
    SolveOut so;
    r = solve(s, so, 1);
    if (r) return r;
    k_transport_update<<<s->L.grd_int, s->L.blk_int, 0, s->st>>>(s->g, dchi, s->md[0], dnew);
    r = launch_check(s, "transport update");
    if (r) return r;
    HIPCHK(s, hipMemcpyAsync(chi_new, dnew, nb, hipMemcpyDeviceToHost, s->st));
    HIPCHK(s, hipStreamSynchronize(s->st));
    if (info) {
        std::memset(info, 0, sizeof(*info));
        double num = 0.0, den = 0.0;
        for (size_t q = 0; q < s->g.n3; ++q) {
            num += (chi_new[q] - chi[q]) * (chi_new[q] - chi[q]);
            den += chi_new[q] * chi_new[q];
        }
        info->res[0] = den > 0.0 ? std::sqrt(num) / std::sqrt(den) : (num == 0.0 ? 0.0 : HUGE_VAL);
        info->relres[0] = so.relres[0];
        info->step = 1;
        info->sweeps[0] = so.sweeps[0];
        info->bicg_iters[0] = so.bicg[0];
        info->omega[0] = s->om[0];
        info->dominance[0] = so.dominance[0];
        info->status = HOSC_OK;
    }
    return HOSC_OK;
}

hosc_status hosc_perf_enable(hosc_solver *s, int32_t on)
{
    if (!s) return HOSC_E_ARG;
    hosc_status r = harvest_events(s);
    if (r) return r;
    if (on && s->ev.empty()) {
        s->ev.resize(2 * kEvPairs);
        s->ev_bytes.resize(kEvPairs);
        s->ev_kind.resize(kEvPairs);
        s->ev_count.resize(kEvPairs);
        for (auto &e : s->ev) HIPCHK(s, hipEventCreate(&e));
    }
    s->prof = on != 0;
    s->perf = hosc_perf{};
    s->ev_used = 0;
    return HOSC_OK;
}

hosc_status hosc_perf_get(hosc_solver *s, hosc_perf *out)
{
    if (!s || !out) return HOSC_E_ARG;
    hosc_status r = harvest_events(s);
    if (r) return r;
    *out = s->perf;
    return HOSC_OK;
}

hosc_status hosc_copy_bandwidth(const void *d_src, void *d_dst, size_t bytes, int32_t reps, hipStream_t stream,
                                double *ms_per_copy)
{
    if (!d_src || !d_dst || !ms_per_copy || reps < 1) return fail(nullptr, HOSC_E_ARG, "invalid copy arguments");
    if (bytes % 16 || reinterpret_cast<uintptr_t>(d_src) % 16 || reinterpret_cast<uintptr_t>(d_dst) % 16)
        return fail(nullptr, HOSC_E_ARG, "copy buffers and size must be 16-byte aligned");
    const size_t n = bytes / 16;
    const int blocks = 256 * 8;    // 8 workgroups of 256 threads per compute unit
    const double2 *src = static_cast<const double2 *>(d_src);
    double2 *dst = static_cast<double2 *>(d_dst);
    const hipError_t e =
        time_launches(stream, reps, [&] { k_copy<<<blocks, 256, 0, stream>>>(src, dst, n); }, ms_per_copy);
    if (e != hipSuccess) return fail(nullptr, HOSC_E_DEVICE, std::string("copy probe: ") + hipGetErrorString(e));
    return HOSC_OK;
}

hosc_status hosc_stream_mix_bandwidth(const void *d_read, void *d_inplace, size_t bytes, int32_t reps,
                                      hipStream_t stream, double *ms_per_launch)
{
    if (!d_read || !d_inplace || !ms_per_launch || reps < 1 || bytes == 0)
        return fail(nullptr, HOSC_E_ARG, "invalid stream-mix probe arguments");
    if (bytes % 16 || reinterpret_cast<uintptr_t>(d_read) % 16 || reinterpret_cast<uintptr_t>(d_inplace) % 16)
        return fail(nullptr, HOSC_E_ARG, "stream-mix probe buffers and size must be 16-byte aligned");
    const size_t n = bytes / 16;
    if ((n + 255) / 256 > 0x7fffffffu) return fail(nullptr, HOSC_E_ARG, "stream-mix probe arrays too long");
    const uintptr_t rd = reinterpret_cast<uintptr_t>(d_read);
    const uintptr_t up = reinterpret_cast<uintptr_t>(d_inplace);
    if (rd < up + (size_t)kMixInPlace * bytes && up < rd + (size_t)kMixRead * bytes)
        return fail(nullptr, HOSC_E_ARG, "stream-mix probe buffers overlap");
    const unsigned blocks = (unsigned)((n + 255) / 256);    // one element of every array per thread
    const double2 *src = static_cast<const double2 *>(d_read);
    double2 *dst = static_cast<double2 *>(d_inplace);
    const hipError_t e =
        time_launches(stream, reps, [&] { k_stream_mix<<<blocks, 256, 0, stream>>>(src, dst, n); }, ms_per_launch);
    if (e != hipSuccess) return fail(nullptr, HOSC_E_DEVICE, std::string("stream-mix probe: ") + hipGetErrorString(e));
    return HOSC_OK;
}

const char *hosc_last_error(const hosc_solver *s)
{
    if (!s) return g_create_error.c_str();
    return s->err.c_str();
}

const char *hosc_status_string(hosc_status st)
{
    switch (st) {
    case HOSC_OK: return "HOSC_OK";
    case HOSC_E_ARG: return "HOSC_E_ARG";
    case HOSC_E_NOMEM: return "HOSC_E_NOMEM";
    case HOSC_E_DEVICE: return "HOSC_E_DEVICE";
    case HOSC_E_NOCONV: return "HOSC_E_NOCONV";
    case HOSC_E_NONFINITE: return "HOSC_E_NONFINITE";
    case HOSC_E_STATE: return "HOSC_E_STATE";
    case HOSC_E_BUDGET: return "HOSC_E_BUDGET";
    }
    return "unknown";
}


hosc_status hosc_batch_workspace_bytes(const hosc_params *p, int32_t count, size_t *bytes)
{
    if (!p || !bytes || count < 1) return bfail(nullptr, HOSC_E_ARG, "params, bytes and count >= 1 are required");
    for (int i = 0; i < count; ++i) {
        const char *e = check_params(&p[i]);
        if (e) return bfail(nullptr, HOSC_E_ARG, "cavity " + std::to_string(i) + ": " + e);
    }
    *bytes = batch_layout(p, count, nullptr);
    return HOSC_OK;
}

hosc_status hosc_batch_create(const hosc_params *p, int32_t count, void *d_ws, size_t ws_bytes, hipStream_t stream,
                              hosc_batch **out)
{
    if (!out) return bfail(nullptr, HOSC_E_ARG, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    hosc_status r = hosc_batch_workspace_bytes(p, count, &need);
    if (r) return r;
    for (int i = 1; i < count; ++i)
        if (p[i].precision != p[0].precision)
            return bfail(nullptr, HOSC_E_ARG, "all cavities of a batch must use one precision");
    if (!d_ws) return bfail(nullptr, HOSC_E_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return bfail(nullptr, HOSC_E_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < need) return bfail(nullptr, HOSC_E_NOMEM, "workspace smaller than hosc_batch_workspace_bytes()");
    hosc_batch *b = new (std::nothrow) hosc_batch();
    if (!b) return bfail(nullptr, HOSC_E_NOMEM, "host allocation failed");
    b->st = stream;
    b->fp32 = p[0].precision == HOSC_FP32_REFINED;
    std::vector<size_t> off;
    batch_layout(p, count, &off);
    char *base = static_cast<char *>(d_ws);
    for (int i = 0; i < count; ++i) {
        hosc_solver *s = nullptr;
        r = hosc_create(&p[i], base + off[i], off[i + 1] - off[i], stream, &s);
        if (r) {
            const std::string msg = "cavity " + std::to_string(i) + ": " + g_create_error;
            for (hosc_solver *x : b->cav) hosc_destroy(x);
            delete b;
            return bfail(nullptr, r, msg);
        }
        b->cav.push_back(s);
    }
    r = fused_init(b->F, count, base + off[count], stream);
    if (r) {
        const std::string msg = b->F.err;
        fused_free(b->F);
        for (hosc_solver *x : b->cav) hosc_destroy(x);
        delete b;
        return bfail(nullptr, r, msg);
    }
    *out = b;
    return HOSC_OK;
}

hosc_status hosc_batch_destroy(hosc_batch *b)
{
    if (!b) return HOSC_OK;
    (void)hipStreamSynchronize(b->st);
    for (int q = 0; q < Fused::kSide; ++q)
        if (b->F.side[q]) (void)hipStreamSynchronize(b->F.side[q]);
    fused_free(b->F);
    for (hosc_solver *s : b->cav) hosc_destroy(s);
    delete b;
    return HOSC_OK;
}

hosc_status hosc_batch_cavity(hosc_batch *b, int32_t idx, hosc_solver **out)
{
    if (!b || !out) return HOSC_E_ARG;
    if (idx < 0 || idx >= (int)b->cav.size()) return bfail(b, HOSC_E_ARG, "cavity index out of range");
    *out = b->cav[idx];
    return HOSC_OK;
}

hosc_status hosc_batch_init_fields(hosc_batch *b, const uint64_t *seeds, double noise_amp)
{
    if (!b || !seeds) return HOSC_E_ARG;
    for (size_t i = 0; i < b->cav.size(); ++i) {
        hosc_status r = hosc_init_fields(b->cav[i], seeds[i], noise_amp);
        if (r) return bfail(b, r, "cavity " + std::to_string(i) + ": " + b->cav[i]->err);
    }
    return HOSC_OK;
}

hosc_status hosc_batch_step(hosc_batch *b, int32_t nsteps, hosc_step_info *info)
{
    if (!b) return HOSC_E_ARG;
    if (nsteps < 0) return bfail(b, HOSC_E_ARG, "nsteps must be >= 0");
    const int n = (int)b->cav.size();
    std::vector<hosc_status> err(n);
    for (int q = 0; q < nsteps; ++q) {
        hosc_status r = fused_step(b->F, b->cav.data(), n, info, err.data());
        if (r) return bfail(b, r, b->F.err);
        for (int i = 0; i < n; ++i)
            if (err[i]) return bfail(b, err[i], "cavity " + std::to_string(i) + ": " + b->cav[i]->err);
    }
    return HOSC_OK;
}

hosc_status hosc_batch_run_to_steady(hosc_batch *b, double res_tol, int64_t max_steps, hosc_step_info *info)
{
    if (!b) return HOSC_E_ARG;
    if (!(res_tol > 0.0)) return bfail(b, HOSC_E_ARG, "res_tol must be > 0");
    if (max_steps < 0) return bfail(b, HOSC_E_ARG, "max_steps must be >= 0");
    const int n = (int)b->cav.size();
    for (int i = 0; i < n; ++i) {
        if (!b->cav[i]->has_state) return bfail(b, HOSC_E_STATE, "cavity " + std::to_string(i) + ": no state set");
        if (b->cav[i]->sticky)
            return bfail(b, HOSC_E_STATE, "cavity " + std::to_string(i) + ": in an error state; set a new state");
    }
    // cavities still marching; each fused step takes only those, so a cavity's
    // arithmetic is that of its single-cavity run whatever the others do
    std::vector<int> running(n, max_steps > 0 ? 1 : 0);
    std::vector<int64_t> taken(n, 0);
    std::vector<hosc_solver *> act;
    std::vector<int> map;
    std::vector<hosc_status> err(n, HOSC_OK);     // indexed by position in act
    std::vector<hosc_step_info> part(n);
    hosc_status first = HOSC_OK;
    std::string msg;
    for (;;) {
        act.clear();
        map.clear();
        for (int i = 0; i < n; ++i)
            if (running[i]) {
                act.push_back(b->cav[i]);
                map.push_back(i);
            }
        if (act.empty()) break;
        const int na = (int)act.size();
        hosc_status r = fused_step(b->F, act.data(), na, part.data(), err.data());
        if (r) return bfail(b, r, b->F.err);
        for (int a = 0; a < na; ++a) {
            const int i = map[a];
            taken[i] += 1;
            if (info) info[i] = part[a];
            if (err[a]) {
                if (!first) {
                    first = err[a];
                    msg = "cavity " + std::to_string(i) + ": " + b->cav[i]->err;
                }
                running[i] = 0;
                continue;
            }
            const double m = std::max(std::max(part[a].res[0], part[a].res[1]), std::max(part[a].res[2], part[a].res[3]));
            if (m < res_tol || taken[i] >= max_steps) running[i] = 0;
        }
    }
    if (first) return bfail(b, first, msg);
    return HOSC_OK;
}

hosc_status hosc_batch_tune(hosc_batch *b, int32_t *grid)
{
    if (!b || !grid) return HOSC_E_ARG;
    for (hosc_solver *s : b->cav)
        if (!s->has_state || s->step != 0)
            return bfail(b, HOSC_E_STATE, "tuning needs every cavity on a freshly set state");
    const int n = (int)b->cav.size();
    int g = 0;
    hosc_status r = b->fp32 ? fused_tune<float>(b->F, b->cav.data(), n, &g) : fused_tune<double>(b->F, b->cav.data(), n, &g);
    if (r) return bfail(b, r, b->F.err);
    *grid = g;
    return HOSC_OK;
}

hosc_status hosc_batch_set_grid(hosc_batch *b, int32_t grid)
{
    if (!b) return HOSC_E_ARG;
    if (grid < 0) return bfail(b, HOSC_E_ARG, "grid must be >= 0");
    b->F.grid = grid;
    return HOSC_OK;
}

hosc_status hosc_batch_perf_enable(hosc_batch *b, int32_t on)
{
    if (!b) return HOSC_E_ARG;
    b->F.prof = on != 0;
    b->F.perf = hosc_perf{};
    return HOSC_OK;
}

hosc_status hosc_batch_perf_get(hosc_batch *b, hosc_perf *out)
{
    if (!b || !out) return HOSC_E_ARG;
    *out = b->F.perf;
    return HOSC_OK;
}

hosc_status hosc_batch_graph_launches(const hosc_batch *b, int64_t *count)
{
    if (!b || !count) return HOSC_E_ARG;
    *count = b->F.graph_launches;
    return HOSC_OK;
}

const char *hosc_batch_last_error(const hosc_batch *b) { return b ? b->err.c_str() : g_create_error.c_str(); }


hosc_status hosc_server_workspace_bytes(size_t hbm_budget_bytes, int32_t max_resident, size_t *bytes)
{
    if (!bytes) return sfail(nullptr, HOSC_E_ARG, "bytes is NULL");
    if (max_resident < 1 || max_resident > 1024) return sfail(nullptr, HOSC_E_ARG, "max_resident must be in [1, 1024]");
    if (hbm_budget_bytes < kAlign) return sfail(nullptr, HOSC_E_ARG, "budget too small");
    *bytes = hbm_budget_bytes / kAlign * kAlign + fused_device_bytes(max_resident);
    return HOSC_OK;
}

hosc_status hosc_server_create(void *d_ws, size_t ws_bytes, size_t hbm_budget_bytes, int32_t max_resident,
                               hipStream_t stream, hosc_server **out)
{
    if (!out) return sfail(nullptr, HOSC_E_ARG, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    hosc_status r = hosc_server_workspace_bytes(hbm_budget_bytes, max_resident, &need);
    if (r) return r;
    if (!d_ws) return sfail(nullptr, HOSC_E_ARG, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return sfail(nullptr, HOSC_E_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < need) return sfail(nullptr, HOSC_E_NOMEM, "workspace smaller than hosc_server_workspace_bytes()");
    hosc_server *v = new (std::nothrow) hosc_server();
    if (!v) return sfail(nullptr, HOSC_E_NOMEM, "host allocation failed");
    v->budget = hbm_budget_bytes / kAlign * kAlign;
    v->max_resident = max_resident;
    v->st = stream;
    v->t0 = std::chrono::steady_clock::now();
    v->arena = static_cast<char *>(d_ws);
    v->d_fused = v->arena + v->budget;
    v->free_[0] = v->budget;
    r = fused_init(v->F, max_resident, v->d_fused, stream);
    v->F.use_graphs = false;    // membership changes every few steps
    if (r) {
        const std::string msg = v->F.err;
        fused_free(v->F);
        delete v;
        return sfail(nullptr, r, msg);
    }
    *out = v;
    return HOSC_OK;
}

hosc_status hosc_server_destroy(hosc_server *v)
{
    if (!v) return HOSC_OK;
    // only the server's own streams are waited for (the stream it was given and its
    // side streams); the caller's other work on the device is not touched
    (void)hipStreamSynchronize(v->st);
    for (int q = 0; q < Fused::kSide; ++q)
        if (v->F.side[q]) (void)hipStreamSynchronize(v->F.side[q]);
    for (auto &r : v->res) hosc_destroy(r.s);
    fused_free(v->F);
    delete v;
    return HOSC_OK;
}

hosc_status hosc_server_now(const hosc_server *v, double *t)
{
    if (!v || !t) return HOSC_E_ARG;
    *t = v->now();
    return HOSC_OK;
}

hosc_status hosc_server_submit(hosc_server *v, const hosc_request *rq, uint64_t *id)
{
    if (!v || !rq) return HOSC_E_ARG;
    const char *e = check_params(&rq->params);
    if (e) return sfail(v, HOSC_E_ARG, e);
    if (!(rq->res_tol > 0.0) || rq->max_steps < 1) return sfail(v, HOSC_E_ARG, "res_tol > 0 and max_steps >= 1 required");
    if (!std::isfinite(rq->noise_amp)) return sfail(v, HOSC_E_ARG, "noise_amp must be finite");
    size_t bytes = 0;
    hosc_status r = hosc_workspace_bytes(&rq->params, &bytes);
    if (r) return sfail(v, r, g_create_error);
    bytes = align_up(bytes);
    if (bytes > v->budget) return sfail(v, HOSC_E_BUDGET, "request workspace exceeds the whole budget");
    hosc_server::Req q;
    q.id = v->next_id++;
    q.rq = *rq;
    if (q.rq.t_arrival < 0.0) q.rq.t_arrival = v->now();
    q.bytes = bytes;
    v->queue.push_back(q);
    if (id) *id = q.id;
    return HOSC_OK;
}

hosc_status hosc_server_step(hosc_server *v, int32_t *resident)
{
    if (!v) return HOSC_E_ARG;
    const double t_in = v->now();
    // admission: first come first served while the head fits
    while (!v->queue.empty() && (int)v->res.size() < v->max_resident) {
        const hosc_server::Req &q = v->queue.front();
        const size_t off = arena_alloc(v, q.bytes);
        if (off == SIZE_MAX) break;
        hosc_solver *s = nullptr;
        hosc_status r = hosc_create(&q.rq.params, v->arena + off, q.bytes, v->st, &s);
        if (!r) r = hosc_init_fields(s, q.rq.seed, q.rq.noise_amp);
        hosc_server::Res rs{q, s, off, v->now(), 0, 0.0};
        v->queue.pop_front();
        v->res.push_back(rs);
        if (r) {
            if (!s) {   // not created: report and release here
                hosc_result out{};
                out.id = rs.q.id;
                out.status = r;
                out.t_arrival = rs.q.rq.t_arrival;
                out.t_admit = out.t_done = v->now();
                v->done.push_back(out);
                arena_free(v, off, rs.q.bytes);
                v->completed += 1;
                v->res.pop_back();
            } else {
                server_retire(v, v->res.size() - 1, r, false);
            }
        }
    }
    if (!v->res.empty()) {
        // one fused step per precision
        for (int prec = 0; prec < 2; ++prec) {
            std::vector<size_t> idx;
            std::vector<hosc_solver *> cav;
            for (size_t k = 0; k < v->res.size(); ++k)
                if ((int)v->res[k].s->fp32 == prec) {
                    idx.push_back(k);
                    cav.push_back(v->res[k].s);
                }
            if (cav.empty()) continue;
            std::vector<hosc_step_info> info(cav.size());
            std::vector<hosc_status> err(cav.size());
            hosc_status r = fused_step(v->F, cav.data(), (int)cav.size(), info.data(), err.data());
            if (r) return sfail(v, r, v->F.err);
            for (size_t a = 0; a < cav.size(); ++a) {
                hosc_server::Res &rs = v->res[idx[a]];
                if (err[a]) continue;
                rs.steps += 1;
                rs.res = std::max(std::max(info[a].res[0], info[a].res[1]), std::max(info[a].res[2], info[a].res[3]));
            }
            v->cavity_steps += (int64_t)cav.size();
            // retire in descending index order (swap-removal keeps lower indices valid)
            for (size_t a = cav.size(); a-- > 0;) {
                hosc_server::Res &rs = v->res[idx[a]];
                if (err[a]) server_retire(v, idx[a], err[a], false);
                else if (rs.res < rs.q.rq.res_tol) server_retire(v, idx[a], HOSC_OK, true);
                else if (rs.steps >= rs.q.rq.max_steps) server_retire(v, idx[a], HOSC_OK, false);
            }
        }
        v->server_steps += 1;
    }
    if (resident) *resident = (int32_t)v->res.size();
    v->busy_s += v->now() - t_in;
    return HOSC_OK;
}

hosc_status hosc_server_poll(hosc_server *v, hosc_result *out, int32_t max, int32_t *n_out)
{
    if (!v || !n_out || (max > 0 && !out)) return HOSC_E_ARG;
    int n = 0;
    while (n < max && !v->done.empty()) {
        out[n++] = v->done.front();
        v->done.pop_front();
    }
    *n_out = n;
    return HOSC_OK;
}

hosc_status hosc_server_stats_get(const hosc_server *v, hosc_server_stats *st)
{
    if (!v || !st) return HOSC_E_ARG;
    st->queued = (int64_t)v->queue.size();
    st->resident = (int64_t)v->res.size();
    st->completed = v->completed;
    st->server_steps = v->server_steps;
    st->cavity_steps = v->cavity_steps;
    st->budget = v->budget;
    st->in_use = v->in_use;
    st->peak = v->peak;
    st->busy_s = v->busy_s;
    return HOSC_OK;
}

const char *hosc_server_last_error(const hosc_server *v) { return v ? v->err.c_str() : g_create_error.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Diagnostics without allocation (hosc_diagnostics_noalloc): every intermediate of
// the Nusselt and entropy reductions lives in one fixed device array of the
// library, sized for N <= kNoAllocMaxN.  In host code `scratch` names a host-side
// stand-in, not the device array: its device address is taken once per device with
// hipGetSymbolAddress, and only that address is ever passed to a kernel.
// ---------------------------------------------------------------------------
namespace {
constexpr int kNoAllocMaxN = 257;
constexpr size_t kNoAllocRound = 32;   // doubles per 256 bytes
constexpr size_t round32(size_t n) { return (n + kNoAllocRound - 1) / kNoAllocRound * kNoAllocRound; }
constexpr size_t kNaN = kNoAllocMaxN;
constexpr size_t kNaOffWq = 0;
constexpr size_t kNaOffAvh = kNaOffWq + round32(kNaN);
constexpr size_t kNaOffAvc = kNaOffAvh + round32(kNaN);
constexpr size_t kNaOffNuh = kNaOffAvc + round32(kNaN);
constexpr size_t kNaOffNuc = kNaOffNuh + round32(kNaN * kNaN);
constexpr size_t kNaOffMx = kNaOffNuc + round32(kNaN * kNaN);
constexpr size_t kNaOffNu = kNaOffMx + round32(kNaN);
constexpr size_t kNaOffEnt = kNaOffNu + round32(8);
constexpr size_t kNaOffPart = kNaOffEnt + round32(8);
// entropy partial sums: 3 per block of the all-node launch (256 nodes per block)
constexpr size_t kNaDoubles = kNaOffPart + round32((kNaN * kNaN * kNaN + 255) / 256 * 3);
}  // namespace

static __device__ __align__(256) double scratch[kNaDoubles];

namespace {
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
double *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device, resolved on the first call there.
hosc_status scratch_on_current_device(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, HOSC_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, HOSC_E_DEVICE, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(nullptr, HOSC_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_dev[dev];
    return HOSC_OK;
}
}  // namespace

extern "C" hosc_status hosc_diagnostics_noalloc(const hosc_params *p, const double *d_u, const double *d_v,
                                                const double *d_w, const double *d_theta, double *d_out,
                                                double *d_nuavg_hot, double *d_nuavg_cold, hipStream_t stream)
{
    const char *err = check_params(p);
    if (err) return fail(nullptr, HOSC_E_ARG, err);
    if (p->N > kNoAllocMaxN)
        return fail(nullptr, HOSC_E_ARG, "N above the no-allocation maximum of " + std::to_string(kNoAllocMaxN));
    if (!d_u || !d_v || !d_w || !d_theta || !d_out)
        return fail(nullptr, HOSC_E_ARG, "d_u, d_v, d_w, d_theta and d_out are required");
    double *base = nullptr;
    hosc_status r = scratch_on_current_device(&base);
    if (r) return r;
    const Geo g = make_geo(p->N);
    const Launch L = make_launch(g);
    Phys ph{};
    ph.Ra = p->Ra;
    ph.Pr = p->Pr;
    ph.dt = p->dt;
    ph.theta_hot = p->theta_hot;
    ph.theta_cold = p->theta_cold;
    ph.theta_ref = p->theta_ref;
    ph.i2_floor = p->i2_floor;
    ph.ex = 0.5 * (p->n_pl - 1.0);
    ph.lambda = p->lambda > 0.0 ? p->lambda : g.h * g.h / (3.0 * p->dt);
    ph.phi = p->phi;
    double *wq = base + kNaOffWq, *nuh = base + kNaOffNuh, *nuc = base + kNaOffNuc;
    double *nu = base + kNaOffNu, *ent = base + kNaOffEnt, *part = base + kNaOffPart, *mxh = base + kNaOffMx;
    double *avh = d_nuavg_hot ? d_nuavg_hot : base + kNaOffAvh;
    double *avc = d_nuavg_cold ? d_nuavg_cold : base + kNaOffAvc;
    const int N = g.N;
    k_simpson_weights<<<(N + 255) / 256, 256, 0, stream>>>(N, wq);
    k_nu_rows<<<N, 256, 0, stream>>>(g, wq, d_theta, nuh, nuc, avh, avc, mxh);
    k_nu_final<<<1, 1024, 0, stream>>>(g, wq, avh, avc, mxh, nu);
    k_entropy<<<L.grd_all, L.blk_all, 0, stream>>>(g, ph, wq, d_u, d_v, d_w, d_theta, nullptr, nullptr, nullptr,
                                                     part);
    k_reduce<<<1, 1024, 0, stream>>>(part, (int)L.nb_all, 3, 0, ent);
    k_diag_pack<<<1, 64, 0, stream>>>(nu, ent, d_out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(nullptr, HOSC_E_DEVICE, std::string("launch of the diagnostics: ") + hipGetErrorString(e));
    return HOSC_OK;
}
