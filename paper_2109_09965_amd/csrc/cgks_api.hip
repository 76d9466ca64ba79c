// C ABI of libcgks.so: batches of cases, device arena layout, uploads and the
// launch sequence of one two-level p-multigrid cycle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "cgks_internal.h"
#include "kernels.h"

using namespace cgks;

namespace {

constexpr int kRedChunk = 1024;   // cells per reduction block (never straddles cases)
constexpr int kMaxGraphCycles = 64;   // cycles one captured graph may hold
constexpr int kMaxColours = 16;   // colours a mesh may use

// First-fit allocator of index ranges in [0, cap): the arena positions of
// one entity type (cells, faces, Gauss points, boundary slots).
struct RangeAlloc {
    int64_t cap = 0;
    std::vector<std::pair<int64_t, int64_t>> free_r;   // (start, length), sorted, coalesced
    std::vector<std::pair<int64_t, int64_t>> used;     // allocated ranges
    void reset(int64_t c) {
        cap = c;
        free_r.clear();
        used.clear();
        if (c > 0) free_r.push_back({0, c});
    }
    int64_t take(int64_t n) {
        if (n == 0) return 0;
        for (size_t k = 0; k < free_r.size(); ++k)
            if (free_r[k].second >= n) {
                const int64_t st = free_r[k].first;
                free_r[k].first += n;
                free_r[k].second -= n;
                if (free_r[k].second == 0) free_r.erase(free_r.begin() + k);
                used.push_back({st, n});
                return st;
            }
        return -1;
    }
    void give(int64_t st, int64_t n) {
        if (n == 0) return;
        for (size_t k = 0; k < used.size(); ++k)
            if (used[k].first == st && used[k].second == n) {
                used.erase(used.begin() + k);
                break;
            }
        free_r.push_back({st, n});
        std::sort(free_r.begin(), free_r.end());
        std::vector<std::pair<int64_t, int64_t>> m;
        for (auto &r : free_r) {
            if (!m.empty() && m.back().first + m.back().second == r.first) m.back().second += r.second;
            else m.push_back(r);
        }
        free_r.swap(m);
    }
    int64_t high_water() const {
        int64_t h = 0;
        for (auto &r : used) h = std::max(h, r.first + r.second);
        return h;
    }
};

struct Arena {
    size_t off = 0;
    template <class T> size_t take(size_t n) {
        off = (off + 255) & ~size_t(255);
        const size_t o = off;
        off += n * sizeof(T) + 0;
        return o;
    }
};

}  // namespace

// A batch is a pool of n_case case slots over an arena with fixed
// capacities NC, NF, NG, NB (cells, faces, Gauss points, boundary slots;
// they are also the strides of the structure-of-arrays fields).  An
// admitted case holds one contiguous range of each entity type for its
// lifetime; kernels launch over the high-water marks and skip entities of
// free slots (case id n_case, never active).
struct cgks_batch {
    int n_case = 0, dim = 0, precision = 0;
    std::vector<const cgks_mesh *> meshes;   // per slot, nullptr when free
    std::vector<cgks_params> params;
    std::vector<char> live;
    int64_t NC = 0, NF = 0, NG = 0, NB = 0;          // capacities
    int64_t hwC = 0, hwF = 0, hwG = 0, hwB = 0;      // launch extents
    RangeAlloc ac, af, ag, ab;
    std::vector<int64_t> cell_off, face_off, gp_base, b_off;
    std::vector<std::pair<const cgks_mesh *, cgks_params>> pending;   // admitted at bind
    int64_t max_rb = 0, max_cb = 0;
    int max_colour = 0;
    // launch shapes (threads per block; cells per sweep block), set by
    // cgks_batch_autotune; results never depend on them
    int blk_flux = kBlock, blk_cell = kBlock, blk_face = kBlock, blk_lcell = kBlock, sweep_chunk = kBlock / 4;
    // sweep blocks per colour
    std::vector<int32_t> cb_start, cb_count;
    std::vector<int64_t> colour_blk_off;   // [max_colour + 1]
    // reduction blocks
    std::vector<int32_t> rb_start, rb_count, rb_case, case_rb_off;
    int n_implicit = 6, n_sweeps = 2, scheme = 0, explicit_only = 0;
    bool any_full = false, any_weno = false;   // some live case uses the full solution / nonlinear weights
    // arena
    size_t bytes = 0;
    char *base = nullptr;
    struct {
        size_t st, ev, Wn, L0, Lt0, G0, geo, vol, h, minv, slot, cell_case;
        size_t fL, fR, fbc, fcase, gp_rng, bslot, avec, S, shift, gavg, bface, gdat;
        size_t gx, gn, gw, fsum, fsum32, ev32, minv32;
        size_t U, Sf, RHS, D, R1, lowf, swp;
        size_t prm, dt, res, force, wallf, case_b, flag, rb_start, rb_count, rb_case, case_rb_off, part0, part1,
            cb_start, cb_count;
        size_t res_hist;
    } o{};
    Dev dev{};
    int32_t *d_cb_start = nullptr, *d_cb_count = nullptr;
    // kernel timing: event pairs recorded around launches
    bool timing = false;
    std::vector<hipEvent_t> events;
    struct TimingRec {
        int kind;
        size_t ev;        // index of the start event; the end event follows
        int launches;     // kernel launches between the two events
    };
    std::vector<TimingRec> recs;
    // captured cycles
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    int graph_cycles = 0;
    double *res_hist = nullptr;                 // device [graph_cycles][n_case], inside the arena
    size_t res_hist_len = 0;
    void drop_graph() {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        graph_exec = nullptr;
        graph = nullptr;
        graph_cycles = 0;
    }
    // pinned host staging of state transfers, grown to the largest case
    double *xfer = nullptr;
    size_t xfer_cap = 0;
    ~cgks_batch() {
        drop_graph();
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        if (xfer) (void)hipHostFree(xfer);
    }
};

namespace {

template <class T> T *at(cgks_batch *b, size_t off) { return reinterpret_cast<T *>(b->base + off); }

void layout(cgks_batch *b) {
    const int d = b->dim, nv = d + 2, nk = ncoef_of(d), nq = nquad_of(d), ns = d == 2 ? 4 : 8;
    const size_t NC = b->NC, NF = b->NF, NG = b->NG, NB = std::max<int64_t>(b->NB, 1);
    Arena a;
    auto &o = b->o;
    const int sr = nv + d * nv, er = d + 1 + nq + nv + nk * nv, gr = d + nq + 1;
    const bool mixed = b->precision != CGKS_FP64;           // FP32 high-order arrays
    const bool ho64 = b->precision != CGKS_MIXED32;         // FP64 high-order arrays
    o.st = a.take<double>(sr * NC);
    o.ev = a.take<double>(ho64 ? er * NC : 0);
    o.Wn = a.take<double>(nv * NC);
    o.L0 = a.take<double>(nv * NC);
    o.Lt0 = a.take<double>(nv * NC);
    o.G0 = a.take<double>(d * nv * NC);
    o.geo = a.take<double>(gr * NC);
    o.vol = a.take<double>(NC);
    o.h = a.take<double>(NC);
    o.minv = a.take<double>(nk * (nk + 1) / 2 * NC);
    o.slot = a.take<int2>(ns * NC);
    o.cell_case = a.take<int32_t>(NC);
    o.fL = a.take<int32_t>(NF);
    o.fR = a.take<int32_t>(NF);
    o.fbc = a.take<int32_t>(NF);
    o.fcase = a.take<int32_t>(NF);
    o.gp_rng = a.take<int2>(NF);
    o.bslot = a.take<int32_t>(NF);
    o.avec = a.take<double>(d * NF);
    o.S = a.take<double>(NF);
    o.shift = a.take<double>(d * NF);
    o.gavg = a.take<double>(nk * NB);
    o.bface = a.take<int32_t>(NB);
    o.gdat = a.take<double>((nv + d * nv) * NB);
    o.gx = a.take<double>(d * NG);
    o.gn = a.take<double>(d * NG);
    o.gw = a.take<double>(NG);
    const int64_t face_rec = 2 * nv + 2 * d * nv;   // Dim<D>::fs
    static_assert(Dim<2>::fs == 2 * 4 + 2 * 2 * 4 && Dim<3>::fs == 2 * 5 + 2 * 3 * 5, "face record size");
    static_assert(Dim<2>::fh + 2 <= Dim<2>::fs && Dim<3>::fh + 3 <= Dim<3>::fs, "planar normal inside the record");
    o.fsum = a.take<double>(ho64 ? face_rec * NF : 0);
    o.fsum32 = a.take<float>(mixed ? face_rec * NF : 0);
    o.ev32 = a.take<float>(mixed ? er * NC : 0);
    o.minv32 = a.take<float>(mixed ? nk * (nk + 1) / 2 * NC : 0);
    // low-level records: U (FP64) + dU (FP64, or FP32 padded to 16 bytes)
    o.U = a.take<double>(size_t(mixed ? (nv + (nv + 1) / 2 + 1) / 2 * 2 : 2 * nv) * NC);
    o.Sf = a.take<double>(nv * NC);
    o.RHS = a.take<double>(nv * NC);
    o.D = a.take<double>(NC);
    o.R1 = a.take<double>(nv * NC);
    o.lowf = a.take<double>(nv * NF);
    o.swp = a.take<double>(4 * NF);
    // per slot, plus the never-active slot n_case that free entities point to
    const size_t K1 = size_t(b->n_case) + 1;
    o.prm = a.take<DevParams>(K1);
    o.dt = a.take<double>(K1);
    o.res = a.take<double>(K1);
    o.force = a.take<double>(3 * K1);
    o.wallf = a.take<double>(3 * NB);
    o.case_b = a.take<int2>(K1);
    o.flag = a.take<int32_t>(K1);
    // table capacities: every case adds at most one partial chunk per block kind
    b->max_rb = int64_t(NC) / kRedChunk + b->n_case + 1;
    // sweep chunks are disjoint and never empty: at most one per cell
    b->max_cb = int64_t(NC) + 1;
    o.rb_start = a.take<int32_t>(b->max_rb);
    o.rb_count = a.take<int32_t>(b->max_rb);
    o.rb_case = a.take<int32_t>(b->max_rb);
    o.case_rb_off = a.take<int32_t>(K1 + 1);
    o.part0 = a.take<double>(b->max_rb);
    o.part1 = a.take<double>(b->max_rb);
    o.cb_start = a.take<int32_t>(b->max_cb);
    o.cb_count = a.take<int32_t>(b->max_cb);
    b->res_hist_len = size_t(kMaxGraphCycles) * b->n_case;
    o.res_hist = a.take<double>(b->res_hist_len);
    b->bytes = (a.off + 255) & ~size_t(255);
}

DevParams dev_params(const cgks_params &p, int dim) {
    DevParams q{};
    q.gamma = p.gamma;
    q.mu = p.mu;
    q.Pr = p.Pr;
    q.T_wall = p.T_wall;
    for (int v = 0; v < 5; ++v) q.W_inf[v] = p.W_inf[v];
    q.cfl_high = p.cfl_high;
    q.cfl_low = p.cfl_low;
    q.dt_fixed = p.dt_fixed;
    q.K = dim == 3 ? (5.0 - 3.0 * p.gamma) / (p.gamma - 1.0) : (4.0 - 2.0 * p.gamma) / (p.gamma - 1.0);
    q.scheme = p.time_scheme;
    q.explicit_only = p.explicit_only;
    q.low_flux = p.low_flux;
    q.flux_full = p.flux_kind == CGKS_FLUX_FULL;
    q.weno_eps = p.weno_eps;
    q.invN = 1.0 / (q.K + dim);
    q.qcoef = (p.Pr != 1.0 && p.mu != 0.0) ? (1.0 / p.Pr - 1.0) * (-p.mu * p.gamma / (p.gamma - 1.0)) : 0.0;
    q.active = 1;
    return q;
}

void fill_dev(cgks_batch *b) {
    auto &o = b->o;
    Dev &d = b->dev;
    d.NC = int32_t(b->NC);
    d.NF = int32_t(b->NF);
    d.NG = int32_t(b->NG);
    d.NB = int32_t(std::max<int64_t>(b->NB, 1));
    d.st = at<double>(b, o.st); d.ev = at<double>(b, o.ev); d.Wn = at<double>(b, o.Wn);
    d.L0 = at<double>(b, o.L0); d.Lt0 = at<double>(b, o.Lt0); d.G0 = at<double>(b, o.G0);
    d.geo = at<double>(b, o.geo);
    d.vol = at<double>(b, o.vol); d.h = at<double>(b, o.h); d.minv = at<double>(b, o.minv);
    d.slot = at<int2>(b, o.slot);
    d.cell_case = at<int32_t>(b, o.cell_case);
    d.fL = at<int32_t>(b, o.fL); d.fR = at<int32_t>(b, o.fR); d.fbc = at<int32_t>(b, o.fbc);
    d.fcase = at<int32_t>(b, o.fcase); d.gp_rng = at<int2>(b, o.gp_rng); d.bslot = at<int32_t>(b, o.bslot);
    d.avec = at<double>(b, o.avec); d.S = at<double>(b, o.S); d.shift = at<double>(b, o.shift);
    d.gavg = at<double>(b, o.gavg);
    d.bface = at<int32_t>(b, o.bface);
    d.gdat = at<double>(b, o.gdat);
    d.NB_real = int32_t(b->hwB);
    d.gx = at<double>(b, o.gx); d.gn = at<double>(b, o.gn); d.gw = at<double>(b, o.gw);
    d.fsum = at<double>(b, o.fsum);
    d.fsum32 = at<float>(b, o.fsum32);
    d.ev32 = at<float>(b, o.ev32);
    d.minv32 = at<float>(b, o.minv32);
    d.U = at<double>(b, o.U); d.Sf = at<double>(b, o.Sf);
    d.RHS = at<double>(b, o.RHS); d.D = at<double>(b, o.D); d.R1 = at<double>(b, o.R1);
    d.lowf = at<double>(b, o.lowf); d.swp = at<double>(b, o.swp);
    d.prm = at<DevParams>(b, o.prm); d.dt = at<double>(b, o.dt); d.res = at<double>(b, o.res);
    d.flag = at<int32_t>(b, o.flag);
    d.force = at<double>(b, o.force); d.case_b = at<int2>(b, o.case_b); d.wallf = at<double>(b, o.wallf);
    d.rb_start = at<int32_t>(b, o.rb_start); d.rb_count = at<int32_t>(b, o.rb_count);
    d.rb_case = at<int32_t>(b, o.rb_case); d.case_rb_off = at<int32_t>(b, o.case_rb_off);
    d.part0 = at<double>(b, o.part0); d.part1 = at<double>(b, o.part1);
    b->d_cb_start = at<int32_t>(b, o.cb_start);
    b->d_cb_count = at<int32_t>(b, o.cb_count);
    b->res_hist = at<double>(b, o.res_hist);
}

template <class T> hipError_t put(cgks_batch *b, size_t off, const std::vector<T> &v, hipStream_t s) {
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(b->base + off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

inline unsigned nblk(int64_t n, int blk = kBlock) { return unsigned((n + blk - 1) / blk); }

// Launch `launch()` (which issues `launches` kernels back to back)
// bracketed by two events when timing is enabled.
template <class F> void timed(cgks_batch *b, int kind, hipStream_t s, F &&launch, int launches = 1) {
    if (!b->timing) {
        launch();
        return;
    }
    const size_t k = b->recs.size() * 2;
    while (b->events.size() < k + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) {
            launch();
            return;
        }
        b->events.push_back(e);
    }
    (void)hipEventRecord(b->events[k], s);
    launch();
    (void)hipEventRecord(b->events[k + 1], s);
    b->recs.push_back({kind, k, launches});
}

#define HIP_TRY(x)                                      \
    do {                                                \
        if ((x) != hipSuccess) return CGKS_EDEVICE;     \
    } while (0)

// the reconstruction and flux kernels in the variant the batch's cases
// need: nonlinear weights and the full gas-kinetic solution are compiled
// into separate instances, so batches without them run the plain kernels
template <int D, typename R> void launch_recon(const cgks_batch *b, const Dev &d, hipStream_t s) {
    const dim3 grid(unsigned((b->hwC + kReconBlock - 1) / kReconBlock));
    if (b->any_weno) hipLaunchKernelGGL((k_recon<D, R, true>), grid, dim3(kReconBlock), 0, s, d);
    else hipLaunchKernelGGL((k_recon<D, R, false>), grid, dim3(kReconBlock), 0, s, d);
}
template <int D, typename R> void launch_flux(const cgks_batch *b, const Dev &d, int blk, int want_grad, hipStream_t s) {
    const dim3 grid(nblk(b->hwF * Dim<D>::lanes, blk));
    if (b->any_full) hipLaunchKernelGGL((k_flux<D, R, true>), grid, dim3(blk), 0, s, d, want_grad);
    else hipLaunchKernelGGL((k_flux<D, R, false>), grid, dim3(blk), 0, s, d, want_grad);
}

template <int D, typename R> void launch_ho_kernels(cgks_batch *b, const Dev &d, int mode, hipStream_t s) {
    timed(b, CGKS_K_RECON, s, [&] {
        if (b->hwB > 0) hipLaunchKernelGGL(k_ghost<D>, dim3(nblk(b->hwB)), dim3(kBlock), 0, s, d);
        launch_recon<D, R>(b, d, s);
    });
    timed(b, CGKS_K_FLUX, s, [&] {
        launch_flux<D, R>(b, d, b->blk_flux, (int)(mode == MODE_R1 ? 0 : mode == MODE_STAGE0 ? 2 : 1), s);
    });
    timed(b, CGKS_K_CELL, s, [&] {
        hipLaunchKernelGGL((k_cell<D, R>), dim3(nblk(b->hwC * Dim<D>::sl, b->blk_cell)), dim3(b->blk_cell), 0, s, d,
                           mode);
    });
}

template <int D> cgks_status launch_highorder(cgks_batch *b, int mode, hipStream_t s) {
    const Dev &d = b->dev;
    if (mode == MODE_STAGE0) {
        timed(b, CGKS_K_DT, s, [&] {
            hipLaunchKernelGGL(k_dt_partial<D>, dim3(b->rb_start.size()), dim3(kBlock), 0, s, d);
            hipLaunchKernelGGL(k_dt_final, dim3(b->n_case), dim3(kBlock), 0, s, d, b->n_case);
        });
    }
    // MIXED32_R64 evaluates the residual pass R1 in FP64
    if (b->precision == CGKS_MIXED32 || (b->precision == CGKS_MIXED32_R64 && mode != MODE_R1))
        launch_ho_kernels<D, float>(b, d, mode, s);
    else launch_ho_kernels<D, double>(b, d, mode, s);
    HIP_TRY(hipGetLastError());
    return CGKS_OK;
}

// ascending then descending colours, n_sweeps times, consecutive repeats of
// a colour dropped (a repeated pass reproduces the same increments)
std::vector<int> sweep_order(int ncol, int nsweeps) {
    std::vector<int> seq;
    for (int sw = 0; sw < nsweeps; ++sw) {
        for (int c = 0; c < ncol; ++c) seq.push_back(c);
        for (int c = ncol - 1; c >= 0; --c) seq.push_back(c);
    }
    std::vector<int> out;
    for (int c : seq)
        if (out.empty() || out.back() != c) out.push_back(c);
    return out;
}

template <int D, typename S> cgks_status launch_lowlevel_s(cgks_batch *b, const double *R1, hipStream_t s) {
    Dev d = b->dev;
    if (R1 != d.R1)
        HIP_TRY(hipMemcpyAsync(d.R1, R1, sizeof(double) * (D + 2) * b->NC, hipMemcpyDeviceToDevice, s));
    timed(b, CGKS_K_LOWFACE, s, [&] {
        hipLaunchKernelGGL((k_low_face<D, S, LOW_SRC_W>), dim3(nblk(b->hwF, b->blk_face)), dim3(b->blk_face), 0, s, d);
    });
    timed(b, CGKS_K_LOWCELL, s, [&] {
        hipLaunchKernelGGL((k_low_cell<D, S, LOW_FORCE>), dim3(nblk(b->hwC * Dim<D>::sl, b->blk_lcell)),
                           dim3(b->blk_lcell), 0, s, d, (double *)nullptr);
    });
    const std::vector<int> order = sweep_order(b->max_colour, b->n_sweeps);
    for (int k = 0; k < b->n_implicit; ++k) {
        // the first step starts at U = W: its set-up came with the forcing
        if (k > 0) {
            timed(b, CGKS_K_LOWFACE, s, [&] {
                hipLaunchKernelGGL((k_low_face<D, S, LOW_SRC_U_DU>), dim3(nblk(b->hwF, b->blk_face)), dim3(b->blk_face), 0, s, d);
            });
            timed(b, CGKS_K_LOWCELL, s, [&] {
                hipLaunchKernelGGL((k_low_cell<D, S, LOW_STEP>), dim3(nblk(b->hwC * Dim<D>::sl, b->blk_lcell)),
                                   dim3(b->blk_lcell), 0, s, d, (double *)nullptr);
            });
        }
        // the colour passes of one step run back to back: one timing span
        int n_pass = 0;
        for (int c : order) n_pass += b->colour_blk_off[c + 1] > b->colour_blk_off[c];
        timed(
            b, CGKS_K_SWEEP, s,
            [&] {
                for (int c : order) {
                    const int64_t b0 = b->colour_blk_off[c], nb = b->colour_blk_off[c + 1] - b0;
                    if (nb == 0) continue;
                    hipLaunchKernelGGL((k_sweep<D, S>), dim3(unsigned(nb)), dim3(4 * b->sweep_chunk), 0, s, d,
                                       (const int32_t *)(b->d_cb_start + b0),
                                       (const int32_t *)(b->d_cb_count + b0));
                }
            },
            n_pass);
    }
    timed(b, CGKS_K_PROLONG, s, [&] {
        hipLaunchKernelGGL((k_prolong_res<D, S>), dim3(b->rb_start.size()), dim3(kBlock), 0, s, d, 1);
        hipLaunchKernelGGL(k_res_final, dim3(b->n_case), dim3(kBlock), 0, s, d, b->n_case);
    });
    HIP_TRY(hipGetLastError());
    return CGKS_OK;
}

// MIXED32 batches run the relaxation sweeps in FP32 (dU stored in FP32)
template <int D> cgks_status launch_lowlevel(cgks_batch *b, const double *R1, hipStream_t s) {
    return b->precision != CGKS_FP64 ? launch_lowlevel_s<D, float>(b, R1, s)
                                     : launch_lowlevel_s<D, double>(b, R1, s);
}

// ---------------------------------------------------------------------
// Scratch of cgks_residual_high_noalloc: the ghost data, reconstruction
// records and face sums of one residual pass live in this array instead of
// the batch arena, for callers that cannot allocate.  Every device the
// library runs on holds its own copy until the process ends.  In host code
// the name stands for a host-side shadow, never a device address: kernels
// receive the address hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices] = {};

// device address of `scratch` on the current device, looked up once per device
cgks_status scratch_address(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CGKS_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return CGKS_EDEVICE;
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return CGKS_OK;
}

// byte offsets of the residual pass's scratch arrays (256-byte aligned) for
// the batch's launch extents; returns the bytes needed
template <int D> size_t scratch_plan(const cgks_batch *b, size_t &o_ev, size_t &o_gd, size_t &o_fs) {
    const size_t rb = b->precision == CGKS_MIXED32 ? sizeof(float) : sizeof(double);
    size_t off = 0;
    auto take = [&off](size_t n) {
        off = (off + 255) & ~size_t(255);
        const size_t o = off;
        off += n;
        return o;
    };
    // the reconstruction stores whole blocks of kReconBlock records (up to NC)
    const int64_t rec_cells = std::min<int64_t>(b->NC, (b->hwC + kReconBlock - 1) / kReconBlock * kReconBlock);
    o_ev = take(size_t(rec_cells) * Rec<D>::er * rb);
    o_gd = take(size_t(std::max<int64_t>(b->hwB, 1)) * (Rec<D>::sr) * sizeof(double));
    // faces beyond the high-water mark belong to no case and store nothing
    o_fs = take(size_t(b->hwF) * Dim<D>::fs * rb);
    return off;
}

template <int D> cgks_status residual_high_noalloc(cgks_batch *b, double *out, hipStream_t s) {
    size_t o_ev = 0, o_gd = 0, o_fs = 0;
    if (scratch_plan<D>(b, o_ev, o_gd, o_fs) > kScratchBytes) return CGKS_ENOMEM;
    void *base = nullptr;
    cgks_status st = scratch_address(&base);
    if (st) return st;
    // the batch's arena must be on the current device (the scratch is per device)
    int dev = -1;
    hipPointerAttribute_t attr{};
    if (hipGetDevice(&dev) != hipSuccess || hipPointerGetAttributes(&attr, b->base) != hipSuccess) return CGKS_EDEVICE;
    if (attr.device != dev) return CGKS_EINVAL;
    char *sb = static_cast<char *>(base);
    Dev d = b->dev;
    d.ev = reinterpret_cast<double *>(sb + o_ev);
    d.ev32 = reinterpret_cast<float *>(sb + o_ev);
    d.gdat = reinterpret_cast<double *>(sb + o_gd);
    d.fsum = reinterpret_cast<double *>(sb + o_fs);
    d.fsum32 = reinterpret_cast<float *>(sb + o_fs);
    d.R1 = out;
    // no timing events here: creating them would allocate
    const bool timing = b->timing;
    b->timing = false;
    if (b->precision == CGKS_MIXED32) launch_ho_kernels<D, float>(b, d, MODE_R1, s);
    else launch_ho_kernels<D, double>(b, d, MODE_R1, s);
    b->timing = timing;
    HIP_TRY(hipGetLastError());
    return CGKS_OK;
}

template <int D> cgks_status launch_cycle(cgks_batch *b, hipStream_t s) {
    cgks_status st = launch_highorder<D>(b, MODE_STAGE0, s);
    if (st) return st;
    if (b->scheme == CGKS_S2O4) {
        st = launch_highorder<D>(b, MODE_STAGE1, s);
        if (st) return st;
    }
    if (b->explicit_only) {
        timed(b, CGKS_K_PROLONG, s, [&] {
            hipLaunchKernelGGL((k_prolong_res<D, double>), dim3(b->rb_start.size()), dim3(kBlock), 0, s, b->dev, 0);
            hipLaunchKernelGGL(k_res_final, dim3(b->n_case), dim3(kBlock), 0, s, b->dev, b->n_case);
        });
        HIP_TRY(hipGetLastError());
        return CGKS_OK;
    }
    st = launch_highorder<D>(b, MODE_R1, s);
    if (st) return st;
    return launch_lowlevel<D>(b, b->dev.R1, s);
}

}  // namespace

extern "C" {

const char *cgks_status_string(cgks_status s) {
    switch (s) {
        case CGKS_OK: return "ok";
        case CGKS_EINVAL: return "invalid argument";
        case CGKS_ENOMEM: return "out of memory or device buffer too small";
        case CGKS_EDEVICE: return "HIP call failed";
        case CGKS_EMESH: return "invalid mesh";
        case CGKS_ENONPHYS: return "non-physical state (density or pressure <= 0)";
        case CGKS_EDIVERGED: return "residual diverged";
        case CGKS_ENOTCONV: return "not converged within max_cycles";
        case CGKS_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

}  // extern "C"

template <class Build> static cgks_status make_mesh(Build &&build, cgks_mesh **out) {
    if (!out) return CGKS_EINVAL;
    *out = nullptr;
    cgks_mesh *m = new (std::nothrow) cgks_mesh;
    if (!m) return CGKS_ENOMEM;
    cgks_status st;
    try {
        st = build(m->hm);
    } catch (const std::bad_alloc &) {
        st = CGKS_ENOMEM;
    }
    if (st != CGKS_OK) {
        delete m;
        return st;
    }
    *out = m;
    return CGKS_OK;
}

extern "C" {

cgks_status cgks_mesh_create(const cgks_mesh_desc *desc, cgks_mesh **out) {
    return make_mesh([desc](HostMesh &hm) { return build_host_mesh_cells(desc, hm); }, out);
}

cgks_status cgks_mesh_create_faces(const cgks_face_mesh_desc *desc, cgks_mesh **out) {
    return make_mesh([desc](HostMesh &hm) { return build_host_mesh(desc, hm); }, out);
}

// planar face: the unit normals of its Gauss points agree with the first
// one's to 1e-12, so its Gauss-Green sums are that normal times one plain
// sum (a change below 1e-12 relative; flat quads whose per-point normals
// differ only by rounding count as planar)
static bool face_planar(const HostMesh &m, int64_t f) {
    const int d = m.dim;
    for (int64_t g = m.gp_off[f] + 1; g < m.gp_off[f + 1]; ++g)
        for (int a = 0; a < d; ++a)
            if (std::fabs(m.gn[g * d + a] - m.gn[m.gp_off[f] * d + a]) > 1e-12) return false;
    return true;
}

cgks_status cgks_mesh_query(const cgks_mesh *mesh, cgks_mesh_info *info) {
    if (!mesh || !info) return CGKS_EINVAL;
    const HostMesh &m = mesh->hm;
    info->dim = m.dim;
    info->n_colour = m.n_colour;
    info->n_cell = m.n_cell;
    info->n_face = m.n_face;
    info->n_gp = m.n_gp;
    info->n_boundary_face = m.n_bface;
    int64_t np = 0;
    for (int64_t f = 0; f < m.n_face; ++f) np += face_planar(m, f) ? 1 : 0;
    info->n_planar_faces = np;
    return CGKS_OK;
}

cgks_status cgks_mesh_permutation(const cgks_mesh *mesh, int64_t *lib_to_caller, int32_t *colour) {
    if (!mesh || !lib_to_caller) return CGKS_EINVAL;
    const HostMesh &m = mesh->hm;
    std::copy(m.lib2caller.begin(), m.lib2caller.end(), lib_to_caller);
    if (colour) std::copy(m.colour.begin(), m.colour.end(), colour);
    return CGKS_OK;
}

cgks_status cgks_mesh_geometry(const cgks_mesh *mesh, double *vol, double *centroid, double *h) {
    if (!mesh) return CGKS_EINVAL;
    const HostMesh &m = mesh->hm;
    if (vol) std::copy(m.vol.begin(), m.vol.end(), vol);
    if (centroid) std::copy(m.ctr.begin(), m.ctr.end(), centroid);
    if (h) std::copy(m.h.begin(), m.h.end(), h);
    return CGKS_OK;
}

cgks_status cgks_mesh_destroy(cgks_mesh *mesh) {
    delete mesh;
    return CGKS_OK;
}

}  // extern "C"

static bool params_ok(const cgks_batch *b, const cgks_params &p) {
    return p.n_implicit == b->n_implicit && p.n_sweeps == b->n_sweeps && p.time_scheme == b->scheme &&
           p.explicit_only == b->explicit_only && p.n_implicit >= 0 && p.n_sweeps >= 0 &&
           (p.time_scheme == CGKS_S2O4 || p.time_scheme == CGKS_S1O2) && p.gamma > 1.0 && p.mu >= 0 && p.Pr > 0 &&
           p.T_wall > 0 && p.cfl_high > 0 && p.cfl_low > 0 && (p.low_flux == CGKS_LOW_KFVS || p.low_flux == CGKS_LOW_LF) &&
           (p.flux_kind == CGKS_FLUX_SMOOTH || p.flux_kind == CGKS_FLUX_FULL) && p.weno_eps >= 0 && p.area_ref >= 0;
}

static cgks_status new_pool(const cgks_pool_desc &q, cgks_batch **out) {
    *out = nullptr;
    if ((q.dim != 2 && q.dim != 3) || q.max_cases <= 0 || q.max_cells <= 0 || q.max_faces <= 0 ||
        q.max_gauss_points <= 0 || q.max_boundary_faces < 0)
        return CGKS_EINVAL;
    if (q.precision != CGKS_FP64 && q.precision != CGKS_MIXED32 && q.precision != CGKS_MIXED32_R64) return CGKS_EINVAL;
    // 32-bit indices: slot tables [8][cells], four lanes per face; face ids
    // + 1 also stay below kSlotPlanar, the planar-face bit of the slot codes
    static_assert(INT32_MAX / 8 + 1 < kSlotPlanar, "face ids must not reach the planar bit");
    if (q.max_cells > INT32_MAX / 8 || q.max_faces > INT32_MAX / 8 || q.max_gauss_points > INT32_MAX / 2 ||
        q.max_boundary_faces > INT32_MAX / 2)
        return CGKS_EINVAL;
    cgks_batch *b = new cgks_batch;
    b->n_case = q.max_cases;
    b->dim = q.dim;
    b->precision = q.precision;
    b->NC = q.max_cells;
    b->NF = q.max_faces;
    b->NG = q.max_gauss_points;
    b->NB = q.max_boundary_faces;
    b->n_implicit = q.n_implicit;
    b->n_sweeps = q.n_sweeps;
    b->scheme = q.time_scheme;
    b->explicit_only = q.explicit_only;
    const size_t K = size_t(q.max_cases);
    b->meshes.assign(K, nullptr);
    b->params.assign(K, cgks_params{});
    b->live.assign(K, 0);
    b->cell_off.assign(K, 0);
    b->face_off.assign(K, 0);
    b->gp_base.assign(K, 0);
    b->b_off.assign(K, 0);
    b->ac.reset(b->NC);
    b->af.reset(b->NF);
    b->ag.reset(b->NG);
    b->ab.reset(b->NB);
    layout(b);
    *out = b;
    return CGKS_OK;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    const int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

static hipError_t fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(nblk(n)), dim3(kBlock), 0, s, p, n, v);
    return hipGetLastError();
}

// strided upload of a structure-of-arrays slice: ncomp rows of n elements
// from host (row pitch n) to field base + off elements (row pitch stride)
template <class T>
static hipError_t put_soa(cgks_batch *b, size_t field, int64_t off, int64_t stride, const std::vector<T> &v,
                          int64_t n, int ncomp, hipStream_t s) {
    if (n == 0) return hipSuccess;
    return hipMemcpy2DAsync(b->base + field + size_t(off) * sizeof(T), size_t(stride) * sizeof(T), v.data(),
                            size_t(n) * sizeof(T), size_t(n) * sizeof(T), size_t(ncomp), hipMemcpyHostToDevice, s);
}
template <class T>
static hipError_t put_at(cgks_batch *b, size_t field, int64_t off, const std::vector<T> &v, hipStream_t s) {
    if (v.empty()) return hipSuccess;
    return hipMemcpyAsync(b->base + field + size_t(off) * sizeof(T), v.data(), v.size() * sizeof(T),
                          hipMemcpyHostToDevice, s);
}

// Geometry, slots and per-slot data of the case in slot c, written into its
// ranges (host tables of that case only); synchronises the stream.
static cgks_status upload_case(cgks_batch *b, int c, hipStream_t s) {
    const HostMesh &m = b->meshes[c]->hm;
    const int d = b->dim, nk = ncoef_of(d), nq = nquad_of(d), ns = d == 2 ? 4 : 8;
    const int nsym = nk * (nk + 1) / 2, gr = d + nq + 1, nv = d + 2;
    const int64_t n = m.n_cell, nf = m.n_face, ng = m.n_gp, nb = m.n_bface;
    const int64_t co = b->cell_off[c], fo = b->face_off[c], go = b->gp_base[c], bo = b->b_off[c];
    std::vector<double> vol(n), h(n), geo(gr * n), minv(nsym * n);
    std::vector<int2> slot(ns * n, make_int2(0, -1));
    std::vector<int32_t> cell_case(n, c);
    std::vector<int32_t> fL(nf), fR(nf), fbc(nf), fcase(nf, c), bslot(nf, -1);
    std::vector<int2> gp_rng(nf);
    std::vector<double> avec(d * nf), S(nf), shift(d * nf), gavg(nk * nb), gx(d * ng), gn(d * ng), gw(ng);
    std::vector<double> swp(4 * nf, 0.0);   // sweep records: area vector now, S lam by each low-level step
    std::vector<int32_t> bface(nb);
    for (int64_t l = 0; l < n; ++l) {
        const int64_t i = m.lib2caller[l];
        vol[l] = m.vol[i];
        h[l] = m.h[i];
        for (int a = 0; a < d; ++a) geo[l * gr + a] = m.ctr[i * d + a];
        for (int q = 0; q < nq; ++q) geo[l * gr + d + q] = m.sec[i * nq + q];
        geo[l * gr + d + nq] = m.h[i];
        int k = 0;
        for (int r = 0; r < nk; ++r)
            for (int t = r; t < nk; ++t) minv[(k++) * n + l] = m.minv[i * nk * nk + r * nk + t];
        int sl = 0;
        for (int64_t q = m.cf_ptr[i]; q < m.cf_ptr[i + 1]; ++q, ++sl) {
            const int64_t f = m.cf_face[q];
            const int side = m.cf_side[q];
            const int64_t nbr = side ? m.owner[f] : m.neigh[f];
            int32_t code = int32_t(fo + m.caller2libf[f] + 1);   // slot order: caller face order
            if (face_planar(m, f)) code |= kSlotPlanar;
            slot[sl * n + l] = make_int2(side ? -code : code, nbr >= 0 ? int32_t(co + m.caller2lib[nbr]) : -1);
        }
    }
    // faces, their Gauss points and boundary slots in the library face order
    int64_t bcount = 0, gl = 0;
    for (int64_t lf = 0; lf < nf; ++lf) {
        const int64_t f = m.libf2caller[lf];
        fL[lf] = int32_t(co + m.caller2lib[m.owner[f]]);
        fR[lf] = m.neigh[f] >= 0 ? int32_t(co + m.caller2lib[m.neigh[f]]) : -1;
        fbc[lf] = m.neigh[f] >= 0 ? 0 : m.bc[f];
        if (face_planar(m, f)) fbc[lf] |= kFacePlanar;
        const int64_t g0 = gl;
        for (int64_t g = m.gp_off[f]; g < m.gp_off[f + 1]; ++g, ++gl) {
            for (int a = 0; a < d; ++a) {
                gx[a * ng + gl] = m.gx[g * d + a];
                gn[a * ng + gl] = m.gn[g * d + a];
            }
            gw[gl] = m.gw[g];
        }
        gp_rng[lf] = make_int2(int32_t(go + g0), int32_t(go + gl));
        for (int a = 0; a < d; ++a) {
            avec[a * nf + lf] = m.avec[f * d + a];
            shift[a * nf + lf] = m.shift[f * d + a];
            swp[4 * lf + a] = m.avec[f * d + a];
        }
        S[lf] = m.S[f];
        if (m.neigh[f] < 0) {
            const int64_t B = bcount++;
            bslot[lf] = int32_t(bo + B);
            bface[B] = int32_t(fo + lf);
            for (int k = 0; k < nk; ++k) gavg[k * nb + B] = m.gavg[f * nk + k];
        }
    }
    auto &o = b->o;
    HIP_TRY(put_at(b, o.vol, co, vol, s)); HIP_TRY(put_at(b, o.h, co, h, s));
    HIP_TRY(put_at(b, o.geo, co * gr, geo, s));
    HIP_TRY(put_soa(b, o.minv, co, b->NC, minv, n, nsym, s));
    if (b->precision != CGKS_FP64) {
        std::vector<float> m32(minv.begin(), minv.end());
        HIP_TRY(put_soa(b, o.minv32, co, b->NC, m32, n, nsym, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    HIP_TRY(put_soa(b, o.slot, co, b->NC, slot, n, ns, s));
    HIP_TRY(put_at(b, o.cell_case, co, cell_case, s));
    HIP_TRY(put_at(b, o.fL, fo, fL, s)); HIP_TRY(put_at(b, o.fR, fo, fR, s)); HIP_TRY(put_at(b, o.fbc, fo, fbc, s));
    HIP_TRY(put_at(b, o.fcase, fo, fcase, s)); HIP_TRY(put_at(b, o.gp_rng, fo, gp_rng, s));
    HIP_TRY(put_at(b, o.bslot, fo, bslot, s));
    HIP_TRY(put_soa(b, o.avec, fo, b->NF, avec, nf, d, s)); HIP_TRY(put_at(b, o.S, fo, S, s));
    HIP_TRY(put_at(b, o.swp, 4 * fo, swp, s));
    HIP_TRY(put_soa(b, o.shift, fo, b->NF, shift, nf, d, s));
    HIP_TRY(put_soa(b, o.gavg, bo, std::max<int64_t>(b->NB, 1), gavg, nb, nk, s));
    HIP_TRY(put_at(b, o.bface, bo, bface, s));
    HIP_TRY(put_soa(b, o.gx, go, b->NG, gx, ng, d, s)); HIP_TRY(put_soa(b, o.gn, go, b->NG, gn, ng, d, s));
    HIP_TRY(put_at(b, o.gw, go, gw, s));
    // per slot; the state and low-level records of the range start at zero
    std::vector<DevParams> prm{dev_params(b->params[c], d)};
    std::vector<double> zero3(3, 0.0), zero1(1, 0.0);
    std::vector<int32_t> zflag(1, 0);
    std::vector<int2> cb{make_int2(int32_t(bo), int32_t(nb))};
    HIP_TRY(put_at(b, o.prm, c, prm, s)); HIP_TRY(put_at(b, o.force, 3 * int64_t(c), zero3, s));
    HIP_TRY(put_at(b, o.dt, c, zero1, s)); HIP_TRY(put_at(b, o.res, c, zero1, s));
    HIP_TRY(put_at(b, o.flag, c, zflag, s)); HIP_TRY(put_at(b, o.case_b, c, cb, s));
    const int sr = nv + d * nv;
    HIP_TRY(hipMemsetAsync(b->base + o.st + size_t(co) * sr * sizeof(double), 0, size_t(n) * sr * sizeof(double), s));
    HIP_TRY(hipStreamSynchronize(s));
    return CGKS_OK;
}

// Sweep chunks (per colour, every live case's runs of that colour), the
// per-case reduction blocks and the launch extents, after the set of live
// cases changed.  Drops a captured graph (its launches have the old shape).
static cgks_status rebuild_tables(cgks_batch *b, hipStream_t s) {
    b->drop_graph();
    b->hwC = b->ac.high_water();
    b->hwF = b->af.high_water();
    b->hwG = b->ag.high_water();
    b->hwB = b->ab.high_water();
    b->dev.NB_real = int32_t(b->hwB);
    b->max_colour = 0;
    b->any_full = b->any_weno = false;
    for (int c = 0; c < b->n_case; ++c)
        if (b->live[c]) {
            b->max_colour = std::max(b->max_colour, b->meshes[c]->hm.n_colour);
            b->any_full = b->any_full || b->params[c].flux_kind == CGKS_FLUX_FULL;
            b->any_weno = b->any_weno || b->params[c].weno_eps > 0;
        }
    b->cb_start.clear();
    b->cb_count.clear();
    b->colour_blk_off.assign(b->max_colour + 1, 0);
    for (int col = 0; col < b->max_colour; ++col) {
        for (int c = 0; c < b->n_case; ++c) {
            if (!b->live[c]) continue;
            const HostMesh &m = b->meshes[c]->hm;
            if (col >= m.n_colour) continue;
            for (int64_t r = m.run_ptr[col]; r < m.run_ptr[col + 1]; ++r) {
                const int64_t start = b->cell_off[c] + m.run_start[r], n = m.run_count[r];
                for (int64_t q = 0; q < n; q += b->sweep_chunk) {
                    b->cb_start.push_back(int32_t(start + q));
                    b->cb_count.push_back(int32_t(std::min<int64_t>(b->sweep_chunk, n - q)));
                }
            }
        }
        b->colour_blk_off[col + 1] = b->cb_start.size();
    }
    b->rb_start.clear();
    b->rb_count.clear();
    b->rb_case.clear();
    b->case_rb_off.assign(1, 0);
    for (int c = 0; c <= b->n_case; ++c) {
        if (c < b->n_case && b->live[c]) {
            const int64_t n = b->meshes[c]->hm.n_cell;
            for (int64_t q = 0; q < n; q += kRedChunk) {
                b->rb_start.push_back(int32_t(b->cell_off[c] + q));
                b->rb_count.push_back(int32_t(std::min<int64_t>(kRedChunk, n - q)));
                b->rb_case.push_back(c);
            }
        }
        b->case_rb_off.push_back(int32_t(b->rb_start.size()));
    }
    if (int64_t(b->cb_start.size()) > b->max_cb || int64_t(b->rb_start.size()) > b->max_rb) return CGKS_EINVAL;
    auto &o = b->o;
    HIP_TRY(put_at(b, o.cb_start, 0, b->cb_start, s)); HIP_TRY(put_at(b, o.cb_count, 0, b->cb_count, s));
    HIP_TRY(put_at(b, o.rb_start, 0, b->rb_start, s)); HIP_TRY(put_at(b, o.rb_count, 0, b->rb_count, s));
    HIP_TRY(put_at(b, o.rb_case, 0, b->rb_case, s)); HIP_TRY(put_at(b, o.case_rb_off, 0, b->case_rb_off, s));
    HIP_TRY(hipStreamSynchronize(s));
    return CGKS_OK;
}

static cgks_status admit(cgks_batch *b, const cgks_mesh *mesh, const cgks_params &p, int c, hipStream_t s) {
    const HostMesh &m = mesh->hm;
    if (m.dim != b->dim || !params_ok(b, p)) return CGKS_EINVAL;
    if (m.n_colour > kMaxColours) return CGKS_EUNSUPPORTED;
    const int64_t co = b->ac.take(m.n_cell);
    const int64_t fo = co < 0 ? -1 : b->af.take(m.n_face);
    const int64_t go = fo < 0 ? -1 : b->ag.take(m.n_gp);
    const int64_t bo = go < 0 ? -1 : b->ab.take(m.n_bface);
    if (bo < 0) {
        if (go >= 0) b->ag.give(go, m.n_gp);
        if (fo >= 0) b->af.give(fo, m.n_face);
        if (co >= 0) b->ac.give(co, m.n_cell);
        return CGKS_ENOMEM;
    }
    b->meshes[c] = mesh;
    b->params[c] = p;
    b->live[c] = 1;
    b->cell_off[c] = co;
    b->face_off[c] = fo;
    b->gp_base[c] = go;
    b->b_off[c] = bo;
    return upload_case(b, c, s);
}

extern "C" {

cgks_status cgks_batch_create(const cgks_mesh *const *meshes, const cgks_params *params, int32_t n_case,
                              int32_t precision, cgks_batch **out) {
    if (!out || !meshes || !params || n_case <= 0) return CGKS_EINVAL;
    *out = nullptr;
    try {
        cgks_pool_desc q{};
        q.dim = meshes[0] ? meshes[0]->hm.dim : 0;
        q.precision = precision;
        q.max_cases = n_case;
        q.n_implicit = params[0].n_implicit;
        q.n_sweeps = params[0].n_sweeps;
        q.time_scheme = params[0].time_scheme;
        q.explicit_only = params[0].explicit_only;
        for (int c = 0; c < n_case; ++c) {
            if (!meshes[c] || meshes[c]->hm.dim != q.dim) return CGKS_EINVAL;
            q.max_cells += meshes[c]->hm.n_cell;
            q.max_faces += meshes[c]->hm.n_face;
            q.max_gauss_points += meshes[c]->hm.n_gp;
            q.max_boundary_faces += meshes[c]->hm.n_bface;
        }
        cgks_batch *b = nullptr;
        cgks_status st = new_pool(q, &b);
        if (st) return st;
        for (int c = 0; c < n_case; ++c) {
            if (!params_ok(b, params[c]) || meshes[c]->hm.n_colour > kMaxColours) {
                delete b;
                return meshes[c]->hm.n_colour > kMaxColours ? CGKS_EUNSUPPORTED : CGKS_EINVAL;
            }
            b->pending.push_back({meshes[c], params[c]});
        }
        *out = b;
    } catch (const std::bad_alloc &) {
        return CGKS_ENOMEM;
    }
    return CGKS_OK;
}

cgks_status cgks_pool_create(const cgks_pool_desc *desc, cgks_batch **out) {
    if (!desc || !out) return CGKS_EINVAL;
    try {
        return new_pool(*desc, out);
    } catch (const std::bad_alloc &) {
        return CGKS_ENOMEM;
    }
}

cgks_status cgks_batch_capacity(const cgks_batch *b, int32_t *max_cases, int64_t *max_cells) {
    if (!b || !max_cases || !max_cells) return CGKS_EINVAL;
    *max_cases = b->n_case;
    *max_cells = b->NC;
    return CGKS_OK;
}

cgks_status cgks_batch_slot_info(const cgks_batch *b, int32_t slot, int32_t *live, int64_t *cell_offset,
                                 int64_t *n_cell) {
    if (!b || slot < 0 || slot >= b->n_case || !live || !cell_offset || !n_cell) return CGKS_EINVAL;
    *live = b->live[slot];
    *cell_offset = b->live[slot] ? b->cell_off[slot] : -1;
    *n_cell = b->live[slot] ? b->meshes[slot]->hm.n_cell : 0;
    return CGKS_OK;
}

cgks_status cgks_batch_query(const cgks_batch *b, size_t *bytes) {
    if (!b || !bytes) return CGKS_EINVAL;
    *bytes = b->bytes;
    return CGKS_OK;
}

cgks_status cgks_batch_bind(cgks_batch *b, void *buf, size_t bytes, void *stream) {
    if (!b || !buf || (reinterpret_cast<uintptr_t>(buf) & 255) || b->base) return CGKS_EINVAL;
    if (bytes < b->bytes) return CGKS_ENOMEM;
    hipStream_t s = static_cast<hipStream_t>(stream);
    b->base = static_cast<char *>(buf);
    fill_dev(b);
    try {
        // everything starts at zero (no slot active); free entities point to
        // the never-active slot n_case, free boundary slots to no face
        HIP_TRY(hipMemsetAsync(b->base, 0, b->bytes, s));
        HIP_TRY(fill_i32(at<int32_t>(b, b->o.cell_case), b->NC, b->n_case, s));
        HIP_TRY(fill_i32(at<int32_t>(b, b->o.fcase), b->NF, b->n_case, s));
        HIP_TRY(fill_i32(at<int32_t>(b, b->o.bface), std::max<int64_t>(b->NB, 1), -1, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (size_t k = 0; k < b->pending.size(); ++k) {
            cgks_status st = admit(b, b->pending[k].first, b->pending[k].second, int(k), s);
            if (st) return st;
        }
        b->pending.clear();
        return rebuild_tables(b, s);
    } catch (const std::bad_alloc &) {
        return CGKS_ENOMEM;
    }
}

cgks_status cgks_batch_admit(cgks_batch *b, const cgks_mesh *mesh, const cgks_params *params, int32_t *slot,
                             void *stream) {
    if (!b || !b->base || !mesh || !params || !slot) return CGKS_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int c = 0;
    while (c < b->n_case && b->live[c]) ++c;
    if (c == b->n_case) return CGKS_ENOMEM;
    try {
        cgks_status st = admit(b, mesh, *params, c, s);
        if (st) return st;
        *slot = c;
        return rebuild_tables(b, s);
    } catch (const std::bad_alloc &) {
        return CGKS_ENOMEM;
    }
}

cgks_status cgks_batch_release(cgks_batch *b, int32_t c, void *stream) {
    if (!b || !b->base || c < 0 || c >= b->n_case || !b->live[c]) return CGKS_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const HostMesh &m = b->meshes[c]->hm;
    // the slot stops running first, then its entities are handed back
    DevParams off{};
    HIP_TRY(hipMemcpyAsync((void *)(b->dev.prm + c), &off, sizeof(DevParams), hipMemcpyHostToDevice, s));
    HIP_TRY(fill_i32(at<int32_t>(b, b->o.cell_case) + b->cell_off[c], m.n_cell, b->n_case, s));
    HIP_TRY(fill_i32(at<int32_t>(b, b->o.fcase) + b->face_off[c], m.n_face, b->n_case, s));
    HIP_TRY(fill_i32(at<int32_t>(b, b->o.bface) + b->b_off[c], m.n_bface, -1, s));
    HIP_TRY(hipStreamSynchronize(s));
    b->ac.give(b->cell_off[c], m.n_cell);
    b->af.give(b->face_off[c], m.n_face);
    b->ag.give(b->gp_base[c], m.n_gp);
    b->ab.give(b->b_off[c], m.n_bface);
    b->live[c] = 0;
    b->meshes[c] = nullptr;
    try {
        return rebuild_tables(b, s);
    } catch (const std::bad_alloc &) {
        return CGKS_ENOMEM;
    }
}

cgks_status cgks_batch_destroy(cgks_batch *b) {
    delete b;
    return CGKS_OK;
}

static cgks_status state_xfer(cgks_batch *b, int32_t c, double *W, double *dW, void *stream, bool up) {
    if (!b || !b->base || c < 0 || c >= b->n_case || !b->live[c] || (up && !W)) return CGKS_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const HostMesh &m = b->meshes[c]->hm;
    const int d = b->dim, nv = d + 2, sr = nv + d * nv;
    const int64_t n = m.n_cell, co = b->cell_off[c];
    const size_t len = size_t(n) * sr;
    if (len > b->xfer_cap) {
        if (b->xfer) (void)hipHostFree(b->xfer);
        b->xfer = nullptr;
        b->xfer_cap = 0;
        HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&b->xfer), len * sizeof(double), hipHostMallocDefault));
        b->xfer_cap = len;
    }
    double *buf = b->xfer;
    double *dev = b->dev.st + size_t(co) * sr;
    // the permutation between caller and library order runs on host threads,
    // each writing its own cells
    if (up) {
        parallel_for(n, [&](int64_t l0, int64_t l1) {
            for (int64_t l = l0; l < l1; ++l) {
                const int64_t i = m.lib2caller[l];
                for (int r = 0; r < nv; ++r) buf[l * sr + r] = W[r * n + i];
                for (int r = 0; r < d * nv; ++r) buf[l * sr + nv + r] = dW ? dW[r * n + i] : 0.0;
            }
        });
        HIP_TRY(hipMemcpyAsync(dev, buf, len * sizeof(double), hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));
        return CGKS_OK;
    }
    HIP_TRY(hipMemcpyAsync(buf, dev, len * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    parallel_for(n, [&](int64_t l0, int64_t l1) {
        for (int64_t l = l0; l < l1; ++l) {
            const int64_t i = m.lib2caller[l];
            if (W)
                for (int r = 0; r < nv; ++r) W[r * n + i] = buf[l * sr + r];
            if (dW)
                for (int r = 0; r < d * nv; ++r) dW[r * n + i] = buf[l * sr + nv + r];
        }
    });
    return CGKS_OK;
}

cgks_status cgks_state_upload(cgks_batch *b, int32_t c, const double *W, const double *dW, void *stream) {
    return state_xfer(b, c, const_cast<double *>(W), const_cast<double *>(dW), stream, true);
}

cgks_status cgks_state_download(cgks_batch *b, int32_t c, double *W, double *dW, void *stream) {
    return state_xfer(b, c, W, dW, stream, false);
}

cgks_status cgks_state_device(cgks_batch *b, int32_t c, double **rec, int32_t *rec_len, int64_t *n_cell) {
    if (!b || !b->base || c < 0 || c >= b->n_case || !b->live[c]) return CGKS_EINVAL;
    const int nv = b->dim + 2, sr = nv + b->dim * nv;
    if (rec) *rec = b->dev.st + size_t(b->cell_off[c]) * sr;
    if (rec_len) *rec_len = sr;
    if (n_cell) *n_cell = b->meshes[c]->hm.n_cell;
    return CGKS_OK;
}

cgks_status cgks_highorder_stage(cgks_batch *b, int32_t stage, void *stream) {
    if (!b || !b->base || stage < 0 || stage > 1 || (stage == 1 && b->scheme != CGKS_S2O4)) return CGKS_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int mode = stage == 0 ? MODE_STAGE0 : MODE_STAGE1;
    return b->dim == 2 ? launch_highorder<2>(b, mode, s) : launch_highorder<3>(b, mode, s);
}

cgks_status cgks_residual(cgks_batch *b, int32_t kind, double *out, void *stream) {
    if (!b || !b->base || !out) return CGKS_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int nv = b->dim + 2;
    if (kind == CGKS_RESIDUAL_HIGH) {
        cgks_status st = b->dim == 2 ? launch_highorder<2>(b, MODE_R1, s) : launch_highorder<3>(b, MODE_R1, s);
        if (st) return st;
        HIP_TRY(hipMemcpyAsync(out, b->dev.R1, sizeof(double) * nv * b->NC, hipMemcpyDeviceToDevice, s));
        return CGKS_OK;
    }
    if (kind == CGKS_RESIDUAL_LOW) {
        if (b->dim == 2) {
            hipLaunchKernelGGL((k_low_face<2, double, LOW_SRC_W>), dim3(nblk(b->hwF)), dim3(kBlock), 0, s, b->dev);
            hipLaunchKernelGGL((k_low_cell<2, double, LOW_R0_OUT>), dim3(nblk(b->hwC * Dim<2>::sl)), dim3(kBlock), 0,
                               s, b->dev, out);
        } else {
            hipLaunchKernelGGL((k_low_face<3, double, LOW_SRC_W>), dim3(nblk(b->hwF)), dim3(kBlock), 0, s, b->dev);
            hipLaunchKernelGGL((k_low_cell<3, double, LOW_R0_OUT>), dim3(nblk(b->hwC * Dim<3>::sl)), dim3(kBlock), 0,
                               s, b->dev, out);
        }
        HIP_TRY(hipGetLastError());
        return CGKS_OK;
    }
    if (kind == CGKS_RESIDUAL_NORM) {
        HIP_TRY(hipMemcpyAsync(out, b->dev.res, sizeof(double) * b->n_case, hipMemcpyDeviceToDevice, s));
        return CGKS_OK;
    }
    return CGKS_EINVAL;
}

cgks_status cgks_residual_high_noalloc(cgks_batch *b, double *out, void *stream) {
    if (!b || !b->base || !out) return CGKS_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return b->dim == 2 ? residual_high_noalloc<2>(b, out, s) : residual_high_noalloc<3>(b, out, s);
}

cgks_status cgks_lowlevel_smooth(cgks_batch *b, const double *R1, void *stream) {
    if (!b || !b->base || !R1) return CGKS_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    return b->dim == 2 ? launch_lowlevel<2>(b, R1, s) : launch_lowlevel<3>(b, R1, s);
}

cgks_status cgks_cycle(cgks_batch *b, double *res, void *stream) {
    if (!b || !b->base) return CGKS_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    cgks_status st = b->dim == 2 ? launch_cycle<2>(b, s) : launch_cycle<3>(b, s);
    if (st) return st;
    if (res) HIP_TRY(hipMemcpyAsync(res, b->dev.res, sizeof(double) * b->n_case, hipMemcpyDeviceToDevice, s));
    return CGKS_OK;
}

cgks_status cgks_solve(cgks_batch *b, const cgks_solve_opts *opts, cgks_solve_report *rep, void *stream) {
    if (!b || !b->base || !opts || !rep || opts->max_cycles <= 0) return CGKS_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int n = b->n_case;
    const int every = std::max(1, opts->check_every);
    std::vector<double> first(n, 0.0);
    std::vector<int32_t> flag(n);
    std::vector<char> done(n, 0);
    int remaining = 0;
    for (int c = 0; c < n; ++c) {
        rep[c] = cgks_solve_report{0, 0, 0.0, 0.0, CGKS_ENOTCONV, {0.0, 0.0, 0.0}, std::nan("")};
        if (b->live[c]) ++remaining;
        else done[c] = 1;   // free slot: nothing to solve
    }
    std::vector<DevParams> prm(n);
    HIP_TRY(hipMemcpyAsync(prm.data(), b->dev.prm, sizeof(DevParams) * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    // blocks of `every` cycles run as one captured graph (one host round trip
    // per block); a shorter final block runs eagerly
    const bool use_graph = every > 1 && every <= 8;
    if (use_graph) {
        cgks_status st = cgks_graph_create(b, every, stream);
        if (st) return st;
    }
    for (int k = 0; k < opts->max_cycles && remaining > 0;) {
        const int todo = std::min(every, opts->max_cycles - k);
        std::vector<double> hist(size_t(todo) * n);
        if (use_graph && todo == every) {
            HIP_TRY(hipGraphLaunch(b->graph_exec, s));
            HIP_TRY(hipMemcpyAsync(hist.data(), b->res_hist, sizeof(double) * todo * n, hipMemcpyDeviceToHost, s));
        } else {
            for (int j = 0; j < todo; ++j) {
                cgks_status st = b->dim == 2 ? launch_cycle<2>(b, s) : launch_cycle<3>(b, s);
                if (st) return st;
                HIP_TRY(hipMemcpyAsync(hist.data() + size_t(j) * n, b->dev.res, sizeof(double) * n,
                                       hipMemcpyDeviceToHost, s));
            }
        }
        HIP_TRY(hipMemcpyAsync(flag.data(), b->dev.flag, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        // every live case ran all `todo` cycles of the block; a stop seen at
        // any of them (or the non-physical flag, known per block only) takes
        // effect at this check, and the report counts the cycles the state ran
        bool changed = false;
        for (int c = 0; c < n; ++c) {
            if (done[c]) continue;
            cgks_status cst = CGKS_OK;
            bool conv = false;
            for (int j = 0; j < todo; ++j) {
                const double r = hist[size_t(j) * n + c];
                const int cyc = k + j + 1;
                if (cyc == 1) rep[c].res_first = first[c] = r;
                if (opts->res_history) opts->res_history[size_t(c) * opts->max_cycles + cyc - 1] = r;
                if (cst != CGKS_OK || conv) continue;
                if (!std::isfinite(r)) cst = CGKS_ENONPHYS;
                else if (r > 1e3 * first[c]) cst = CGKS_EDIVERGED;
                else conv = opts->tol_abs ? r <= opts->tol : (first[c] > 0 && r / first[c] <= opts->tol);
            }
            if (cst == CGKS_OK && (flag[c] & 1)) cst = CGKS_ENONPHYS;
            rep[c].cycles = k + todo;
            rep[c].res_last = hist[size_t(todo - 1) * n + c];
            if (cst != CGKS_OK || conv) {
                done[c] = 1;
                --remaining;
                rep[c].converged = conv && cst == CGKS_OK;
                rep[c].status = cst;
                prm[c].active = 0;
                changed = true;
            }
        }
        if (changed) {
            HIP_TRY(hipMemcpyAsync((void *)b->dev.prm, prm.data(), sizeof(DevParams) * n, hipMemcpyHostToDevice, s));
            HIP_TRY(hipStreamSynchronize(s));
        }
        k += todo;
    }
    // leave every admitted case active again for later calls
    for (int c = 0; c < n; ++c) prm[c].active = b->live[c] ? 1 : 0;
    HIP_TRY(hipMemcpyAsync((void *)b->dev.prm, prm.data(), sizeof(DevParams) * n, hipMemcpyHostToDevice, s));
    // wall force of each case's last stage-0 pass (a frozen case kept its
    // wall sums from its last active cycle)
    std::vector<double> force(3 * size_t(n)), cd(n);
    {
        cgks_status fst = cgks_wall_force(b, force.data(), cd.data(), stream);
        if (fst) return fst;
    }
    for (int c = 0; c < n; ++c) {
        for (int a = 0; a < 3; ++a) rep[c].force[a] = force[3 * size_t(c) + a];
        rep[c].cd = cd[c];
    }
    return CGKS_OK;
}

cgks_status cgks_wall_force(cgks_batch *b, double *force, double *cd, void *stream) {
    if (!b || !b->base || !force) return CGKS_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (b->hwB > 0) {
        if (b->dim == 2) hipLaunchKernelGGL(k_wall_force<2>, dim3(b->n_case), dim3(kBlock), 0, s, b->dev);
        else hipLaunchKernelGGL(k_wall_force<3>, dim3(b->n_case), dim3(kBlock), 0, s, b->dev);
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipMemcpyAsync(force, b->dev.force, sizeof(double) * 3 * b->n_case, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (cd) {
        // Cd = F . e_inf / (1/2 rho_inf |U_inf|^2 A_ref), e_inf = U_inf / |U_inf|
        for (int c = 0; c < b->n_case; ++c) {
            cd[c] = std::nan("");
            if (!b->live[c]) continue;
            const cgks_params &p = b->params[c];
            const double rho = p.W_inf[0];
            double u2 = 0, fu = 0;
            for (int a = 0; a < b->dim; ++a) {
                const double u = p.W_inf[1 + a] / rho;
                u2 += u * u;
                fu += force[3 * size_t(c) + a] * u;
            }
            if (p.area_ref > 0 && u2 > 0) cd[c] = fu / std::sqrt(u2) / (0.5 * rho * u2 * p.area_ref);
        }
    }
    return CGKS_OK;
}

}  // extern "C"

// Times the candidate launch shapes of the face, cell and sweep kernels on
// the batch's own data and keeps the fastest.  Only launches that leave the
// state W, grad W untouched are timed: the reconstruction from the current
// state, the flux with gradient sums, the residual pass of k_cell, the
// low-level face flux and R0, and whole sequences of colour passes on the
// low-level work arrays (set up from the current state first).
template <int D, typename R, typename S> static cgks_status autotune_t(cgks_batch *b, hipStream_t s) {
    const Dev &d = b->dev;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    auto time_of = [&](auto &&launch) -> float {
        launch();                     // warm-up
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < 5; ++r) launch();
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        return ms;
    };
    // cand[0] is the default shape; another one is taken only when it is
    // at least 3 % faster (timing noise must not move the choice)
    auto pick = [&](const int *cand, int n, auto &&launch_with) {
        int best = cand[0];
        const float t0 = time_of([&] { launch_with(cand[0]); });
        float bt = t0;
        for (int k = 1; k < n; ++k) {
            const float t = time_of([&] { launch_with(cand[k]); });
            if (t < bt && t < 0.97f * t0) bt = t, best = cand[k];
        }
        return best;
    };
    static const int blocks[3] = {256, 128, 64};
    if (b->hwB > 0) hipLaunchKernelGGL(k_ghost<D>, dim3(nblk(b->hwB)), dim3(kBlock), 0, s, d);
    launch_recon<D, R>(b, d, s);
    b->blk_flux = pick(blocks, 3, [&](int blk) { launch_flux<D, R>(b, d, blk, 1, s); });
    b->blk_cell = pick(blocks, 3, [&](int blk) {
        hipLaunchKernelGGL((k_cell<D, R>), dim3(nblk(b->hwC * Dim<D>::sl, blk)), dim3(blk), 0, s, d, (int)MODE_R1);
    });
    b->blk_face = pick(blocks, 3, [&](int blk) {
        hipLaunchKernelGGL((k_low_face<D, S, LOW_SRC_W>), dim3(nblk(b->hwF, blk)), dim3(blk), 0, s, d);
    });
    b->blk_lcell = pick(blocks, 3, [&](int blk) {
        hipLaunchKernelGGL((k_low_cell<D, S, LOW_R0_OUT>), dim3(nblk(b->hwC * Dim<D>::sl, blk)), dim3(blk), 0, s, d,
                           d.Sf);
    });
    // low-level work arrays from the current state, then the sweep chunk
    hipLaunchKernelGGL((k_low_face<D, S, LOW_SRC_W>), dim3(nblk(b->hwF, b->blk_face)), dim3(b->blk_face), 0, s, d);
    hipLaunchKernelGGL((k_low_cell<D, S, LOW_FORCE>), dim3(nblk(b->hwC * Dim<D>::sl, b->blk_lcell)), dim3(b->blk_lcell),
                       0, s, d, (double *)nullptr);
    static const int chunks[3] = {64, 32, 16};
    cgks_status st = CGKS_OK;
    const std::vector<int> order = sweep_order(b->max_colour, b->n_sweeps);
    const int chunk = pick(chunks, 3, [&](int ch) {
        if (b->sweep_chunk != ch) {
            b->sweep_chunk = ch;
            if (rebuild_tables(b, s) != CGKS_OK) st = CGKS_EDEVICE;
        }
        for (int c : order) {   // the colour passes of one implicit step
            const int64_t b0 = b->colour_blk_off[c], nb = b->colour_blk_off[c + 1] - b0;
            if (nb == 0) continue;
            hipLaunchKernelGGL((k_sweep<D, S>), dim3(unsigned(nb)), dim3(4 * ch), 0, s, d,
                               (const int32_t *)(b->d_cb_start + b0), (const int32_t *)(b->d_cb_count + b0));
        }
    });
    b->sweep_chunk = chunk;
    if (st == CGKS_OK) st = rebuild_tables(b, s);
    // nothing the timing did counts as a health event
    std::vector<int32_t> zero(b->n_case + 1, 0);
    HIP_TRY(hipMemcpyAsync(b->dev.flag, zero.data(), sizeof(int32_t) * zero.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIP_TRY(hipGetLastError());
    return st;
}

extern "C" {

cgks_status cgks_batch_autotune(cgks_batch *b, int32_t *choice, void *stream) {
    if (!b || !b->base) return CGKS_EINVAL;
    bool any = false;
    for (int c = 0; c < b->n_case; ++c) any |= b->live[c] != 0;
    if (!any) return CGKS_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    b->drop_graph();
    cgks_status st;
    const bool f32 = b->precision != CGKS_FP64;
    if (b->dim == 2) st = f32 ? autotune_t<2, float, float>(b, s) : autotune_t<2, double, double>(b, s);
    else st = f32 ? autotune_t<3, float, float>(b, s) : autotune_t<3, double, double>(b, s);
    if (st) return st;
    if (choice) {
        choice[0] = b->blk_flux;
        choice[1] = b->blk_cell;
        choice[2] = b->blk_face;
        choice[3] = b->blk_lcell;
        choice[4] = b->sweep_chunk;
    }
    return CGKS_OK;
}

cgks_status cgks_graph_create(cgks_batch *b, int32_t n_cycles, void *stream) {
    if (!b || !b->base || n_cycles <= 0 || n_cycles > kMaxGraphCycles) return CGKS_EINVAL;
    b->drop_graph();
    hipStream_t cap;
    HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    // the capture stream starts after all work already queued on `stream`
    hipEvent_t ready;
    HIP_TRY(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(ready, static_cast<hipStream_t>(stream)));
    HIP_TRY(hipStreamWaitEvent(cap, ready, 0));
    HIP_TRY(hipStreamSynchronize(cap));
    const bool timing = b->timing;
    b->timing = false;
    cgks_status st = CGKS_OK;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) st = CGKS_EDEVICE;
    for (int k = 0; k < n_cycles && st == CGKS_OK; ++k) {
        st = b->dim == 2 ? launch_cycle<2>(b, cap) : launch_cycle<3>(b, cap);
        if (st == CGKS_OK)
            hipLaunchKernelGGL(k_res_store, dim3(nblk(b->n_case)), dim3(kBlock), 0, cap, (const double *)b->dev.res,
                               b->res_hist + size_t(k) * b->n_case, b->n_case);
    }
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cap, &g);
    b->timing = timing;
    if (st == CGKS_OK && (e != hipSuccess || !g)) st = CGKS_EDEVICE;
    if (st == CGKS_OK && hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) st = CGKS_EDEVICE;
    if (st == CGKS_OK) {
        b->graph = g;
        b->graph_cycles = n_cycles;
    } else if (g) {
        (void)hipGraphDestroy(g);
    }
    (void)hipEventDestroy(ready);
    (void)hipStreamDestroy(cap);
    return st;
}

cgks_status cgks_graph_launch(cgks_batch *b, double *res_history_dev, void *stream) {
    if (!b || !b->graph_exec) return CGKS_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipGraphLaunch(b->graph_exec, s));
    if (res_history_dev)
        HIP_TRY(hipMemcpyAsync(res_history_dev, b->res_hist, sizeof(double) * b->graph_cycles * b->n_case,
                               hipMemcpyDeviceToDevice, s));
    return CGKS_OK;
}

cgks_status cgks_graph_destroy(cgks_batch *b) {
    if (!b) return CGKS_EINVAL;
    b->drop_graph();
    return CGKS_OK;
}

cgks_status cgks_timing_enable(cgks_batch *b, int32_t enable) {
    if (!b) return CGKS_EINVAL;
    b->timing = enable != 0;
    b->recs.clear();
    return CGKS_OK;
}

cgks_status cgks_timing_read(cgks_batch *b, double *ms, int64_t *launches) {
    if (!b || !ms || !launches) return CGKS_EINVAL;
    for (int k = 0; k < CGKS_KERNEL_KINDS; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (auto &r : b->recs) {
        HIP_TRY(hipEventSynchronize(b->events[r.ev + 1]));
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, b->events[r.ev], b->events[r.ev + 1]));
        ms[r.kind] += t;
        launches[r.kind] += r.launches;
    }
    b->recs.clear();
    return CGKS_OK;
}

}  // extern "C"
