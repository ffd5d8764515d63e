// Batched solves: many Algorithm 3 instances (Sec. 4) of uneven size in one
// persistent launch.
//
// The launch is split into groups of workgroups.  Each group runs an ordered
// list of instances one after the other, every instance on the group's whole
// sub-grid with its own barrier area and work blocks, so groups never wait
// for each other.  The host picks the group sizes and lists from a cost model
// of one Taylor term (exchange latency plus the rounds of rows each thread
// works through) and the expected term count of each instance (s_int steps of
// the Taylor length that tol implies), minimising the predicted makespan: an
// instance that alone needs more than the makespan gets a group of several
// workgroups, the rest are packed longest-first onto single workgroups.
// The launch (barrier reset and solve kernel) is captured once into a HIP
// graph and replayed by every run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "batch_kernel.h"

using namespace phc;

namespace phc {

// Resets every instance's barrier area and status words (one block each).
__global__ void batch_sync_init(const SolveArgs *__restrict__ args, int count) {
    const int it = blockIdx.x;
    if (it >= count)
        return;
    unsigned *bar = args[it].bar;
    for (int i = threadIdx.x; i < kSyncLines * kLineU; i += blockDim.x)
        bar[i] = 0u;
    if (threadIdx.x < 8)
        args[it].info[threadIdx.x] = 0;
}

static BatchKernel pick_batch_kernel(int kind, bool mix) {
    if (kind == kStencil)
        return batch_kernel_stencil(mix);
    if (kind == kCsr)
        return batch_kernel_csr(mix);
    return nullptr;
}

// ------------------------------------------------------------ cost model
// Terms of one Taylor loop at tolerance tol: the scaled step has norm about
// theta = (tol m!)^(1/m) (m = 61, Sec. 3), and the loop runs until
// theta^k / k! drops below tol.
static double taylor_terms(double tol) {
    const double m = 61.0;
    const double lt = std::log(std::max(tol, 1e-300));
    const double theta = std::exp((lt + std::lgamma(m + 1.0)) / m);
    const double lth = std::log(theta);
    int k = 1;
    while (k < kTermCap && (k * lth - std::lgamma(k + 1.0)) > lt)
        ++k;
    return (double)k + 1.0;
}

struct ItemCost {
    double terms;   // Taylor terms over the whole solve
    double cols;    // columns of the recovery block (2r)
    int64_t n;
    int gmax;       // most workgroups that still own 512 rows each
};

// One term on G workgroups, microseconds: the exchange (a workgroup barrier
// for G = 1, the grid barrier otherwise, growing with G) plus the rounds of
// rows each thread works through one after another, ceil(n / (512 G)), each
// taking a latency that grows with the block's width.  A term is bound by
// memory latency per round rather than by bytes per CU at these sizes.  The
// starting constants are MI355X measurements; every run of a plan refits
// them from the device clocks of its instances (least squares over the
// instances), and the autotuner keeps the fitted model on disk.
struct Model {
    double e1 = 1.5;     // single-workgroup exchange (us)
    double e2 = 2.1;     // grid exchange (us)
    double g2 = 0.021;   // growth of the grid exchange per workgroup (us)
    double l0 = 0.05;    // one round of rows (us)
    double l1 = 1.27;    // one round of rows, per column (us)
};
static thread_local Model t_model;

static double rounds(const ItemCost &c, int G) {
    return std::ceil((double)c.n / ((double)kNT * (double)G));
}
static double term_us(const ItemCost &c, int G) {
    const Model &m = t_model;
    const double ex = (G == 1) ? m.e1 : m.e2 + m.g2 * G;
    return ex + rounds(c, G) * (m.l0 + m.l1 * c.cols);
}
static double cost_us(const ItemCost &c, int G) { return c.terms * term_us(c, G); }

constexpr int kExplore = 3;   // refit plans a batch tries before keeping its best

struct Schedule {
    std::vector<int> gsize;                 // per group
    std::vector<std::vector<int>> glist;    // per group, instance order
    double makespan = 0.0;
    int wgs = 0;
};

// Smallest predicted makespan M with a schedule of at most cap workgroups:
// every instance, longest first, gets the fewest workgroups that finish it
// within M, and joins the smallest existing group of at least that size that
// still finishes within M (first fit), else opens a group of its own.  A
// group runs its instances one after another, so a workgroup that an early
// instance leaves idle takes later ones instead of waiting for the launch end.
static bool schedule_for(const std::vector<ItemCost> &c, int cap, double M, Schedule &out) {
    const int count = (int)c.size();
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(),
              [&](int a, int b) { return cost_us(c[a], 1) > cost_us(c[b], 1); });
    Schedule s;
    std::vector<double> load;   // per group
    for (int it : order) {
        int G = 1;
        while (G < c[it].gmax && cost_us(c[it], G) > M)
            ++G;
        if (cost_us(c[it], G) > M)
            return false;   // cannot meet M even with every useful workgroup
        int best = -1;
        for (size_t g = 0; g < s.gsize.size(); ++g) {
            const int gs = s.gsize[g];
            if (gs < G || (best >= 0 && gs >= s.gsize[best]))
                continue;
            if (load[g] + cost_us(c[it], gs) <= M)
                best = (int)g;
        }
        if (best < 0) {
            s.gsize.push_back(G);
            s.glist.push_back({});
            load.push_back(0.0);
            s.wgs += G;
            if (s.wgs > cap)
                return false;
            best = (int)s.gsize.size() - 1;
        }
        load[best] += cost_us(c[it], s.gsize[best]);
        s.glist[best].push_back(it);
    }
    if (s.wgs > cap)
        return false;
    double mk = 0.0;
    for (size_t g = 0; g < s.gsize.size(); ++g) {
        double t = 0.0;
        for (int it : s.glist[g])
            t += cost_us(c[it], s.gsize[g]);
        mk = std::max(mk, t);
    }
    s.makespan = mk;
    out = std::move(s);
    return true;
}

static Schedule make_schedule(const std::vector<ItemCost> &c, int cap) {
    double lo = 0.0, hi = 0.0;
    for (const auto &x : c)
        hi += cost_us(x, 1);
    hi = std::max(hi, 1.0);
    Schedule best;
    if (!schedule_for(c, cap, hi, best)) {
        // more instances than workgroups with everything on one: one group per
        // workgroup, instances dealt longest-first
        best = Schedule();
        const int ng = std::min<int>(cap, (int)c.size());
        best.gsize.assign(ng, 1);
        best.glist.assign(ng, {});
        std::vector<double> load(ng, 0.0);
        std::vector<int> order(c.size());
        std::iota(order.begin(), order.end(), 0);
        std::sort(order.begin(), order.end(),
                  [&](int a, int b) { return cost_us(c[a], 1) > cost_us(c[b], 1); });
        for (int it : order) {
            const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            load[k] += cost_us(c[it], 1);
            best.glist[k].push_back(it);
        }
        best.wgs = ng;
        best.makespan = *std::max_element(load.begin(), load.end());
        return best;
    }
    for (int iter = 0; iter < 60; ++iter) {
        const double mid = 0.5 * (lo + hi);
        Schedule s;
        if (schedule_for(c, cap, mid, s)) {
            best = std::move(s);
            hi = mid;
        } else {
            lo = mid;
        }
        if (hi - lo < 1e-3 * hi)
            break;
    }
    return best;
}

}  // namespace phc

struct phicomb_batch_s {
    int device = 0;
    int count = 0;
    int kind = 0;
    int precision = 0;
    bool mix = false;
    int runs = 0;                 // runs whose clocks refit the model
    int explored = 0;             // plans tried after a refit
    double best_ms = 0.0;         // fastest measured launch and its schedule
    Schedule best_sched;
    double last_measured_ms = 0.0, last_predicted_ms = 0.0, refit_predicted_ms = 0.0;
    int cap = 0;                  // workgroups the launch may use
    std::vector<phicomb_op> ops;
    std::vector<int> p, r, s_int;
    std::vector<ItemCost> cost;
    Model model;
    Schedule sched;
    int wgs = 0;
    int ng = 0;
    void *mem = nullptr;          // device: args, tables, status words, clocks, work blocks
    SolveArgs *args = nullptr;
    int *tables = nullptr;        // variant, wg_group, gfirst, gsize, goff, glist
    int *info_dev = nullptr;      // [count][8], gathered after the solve
    long long *ts_dev = nullptr;  // [count][2] wall clock at start / end of every instance
    int *info_host = nullptr;     // pinned copies
    long long *ts_host = nullptr;
    double clock_khz = 0.0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool no_graph = false;
    BatchKernel kernel = nullptr;
};

namespace {

__global__ void batch_gather_info(const SolveArgs *__restrict__ args, int *__restrict__ out,
                                  int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count * 8)
        out[i] = args[i / 8].info[i % 8];
}

void drop_graph(phicomb_batch b) {
    if (b->exec)
        hipGraphExecDestroy(b->exec);
    if (b->graph)
        hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

void free_batch(phicomb_batch b) {
    if (!b)
        return;
    drop_graph(b);
    if (b->cap_stream)
        hipStreamDestroy(b->cap_stream);
    if (b->mem)
        hipFree(b->mem);
    if (b->info_host)
        hipHostFree(b->info_host);
    if (b->ts_host)
        hipHostFree(b->ts_host);
    delete b;
}

size_t table_ints(int count, int cap) { return (size_t)2 * count + cap + 3 * (size_t)cap + 1; }

// Schedule with the plan's model, then the launch tables (the layout of an
// instance depends on the size of its group).  Drops the captured graph.
int build_plan(phicomb_batch b, const Schedule *use = nullptr) {
    t_model = b->model;
    b->sched = use ? *use : make_schedule(b->cost, b->cap);
    b->wgs = b->sched.wgs;
    b->ng = (int)b->sched.gsize.size();
    const int count = b->count, ng = b->ng;
    std::vector<int> tab(table_ints(count, b->cap), 0);
    int *t_variant = tab.data();
    int *t_wg = t_variant + count;
    int *t_gfirst = t_wg + b->wgs;
    int *t_gsize = t_gfirst + ng;
    int *t_goff = t_gsize + ng;
    int *t_glist = t_goff + ng + 1;
    int wg = 0, lo = 0;
    for (int g = 0; g < ng; ++g) {
        const int G = b->sched.gsize[g];
        t_gfirst[g] = wg;
        t_gsize[g] = G;
        for (int k = 0; k < G; ++k)
            t_wg[wg++] = g;
        t_goff[g] = lo;
        for (int it : b->sched.glist[g]) {
            t_glist[lo++] = it;
            const int64_t n = b->cost[it].n;
            const int64_t rpt = (n + (int64_t)kNT * G - 1) / ((int64_t)kNT * G);
            const int layout = rpt <= 1 ? 0 : rpt <= 2 ? 1 : rpt <= 4 ? 2 : kLayoutEmem;
            t_variant[it] = (b->r[it] - 1) * kLayouts + layout;
        }
    }
    t_goff[ng] = lo;
    drop_graph(b);
    if (hipMemcpy(b->tables, tab.data(), sizeof(int) * tab.size(), hipMemcpyHostToDevice) !=
        hipSuccess)
        return PHICOMB_EDEVICE;
    return PHICOMB_OK;
}

// The model's constants from per-instance samples (workgroups G, rounds,
// columns, measured microseconds per term), in two stages so that every
// constant stays physical: the per-round constants (l0, l1) by least squares
// over the samples whose rounds dominate (4 or more rounds), then the
// exchange constants from what remains: e1 the mean remainder of the
// single-workgroup samples of at most 4 rounds, (e2, g2) a least-squares
// line in G through the remainders of the grid samples of at most 2 rounds
// (where the exchange is a large part of a term).  Constants without samples
// keep their values; all are clamped to small positive floors.  The defaults
// are such a fit to the device clocks of the 256-instance benchmark batch.
struct Sample {
    double G, rounds, cols, us, terms;
};

// Weighted least squares for y ~ a x1 + b x2 (weights w).
static bool lsq2(const std::vector<double> &x1, const std::vector<double> &x2,
                 const std::vector<double> &y, const std::vector<double> &w, double &a,
                 double &b) {
    double s11 = 0, s12 = 0, s22 = 0, s1y = 0, s2y = 0;
    for (size_t k = 0; k < y.size(); ++k) {
        s11 += w[k] * x1[k] * x1[k];
        s12 += w[k] * x1[k] * x2[k];
        s22 += w[k] * x2[k] * x2[k];
        s1y += w[k] * x1[k] * y[k];
        s2y += w[k] * x2[k] * y[k];
    }
    const double det = s11 * s22 - s12 * s12;
    if (y.size() < 3 || !(std::fabs(det) > 1e-12 * (s11 * s22 + 1e-300)))
        return false;
    a = (s1y * s22 - s2y * s12) / det;
    b = (s2y * s11 - s1y * s12) / det;
    return std::isfinite(a) && std::isfinite(b);
}

// Every sample is weighted by its term count: the fit then matches the
// instances that hold the launch's time (a few long chains), not the many
// short ones whose per-term time is dominated by their few S-series terms.
bool fit_model(const std::vector<Sample> &smp, Model &m) {
    Model out = m;
    {
        std::vector<double> x1, x2, y, w;
        for (const Sample &s : smp)
            if (s.rounds >= 4.0) {
                x1.push_back(s.rounds);
                x2.push_back(s.rounds * s.cols);
                y.push_back(s.us);
                w.push_back(s.terms);
            }
        double a, b;
        if (lsq2(x1, x2, y, w, a, b)) {
            out.l0 = std::max(a, 0.05);
            out.l1 = std::max(b, 0.05);
        }
    }
    double r1 = 0.0, w1 = 0.0;
    std::vector<double> r2, g2, w2;
    for (const Sample &s : smp) {
        const double rest = s.us - s.rounds * (out.l0 + out.l1 * s.cols);
        if (s.G == 1.0 && s.rounds <= 4.0) {
            r1 += s.terms * rest;
            w1 += s.terms;
        } else if (s.G > 1.0 && s.rounds <= 2.0) {
            r2.push_back(rest);
            g2.push_back(s.G);
            w2.push_back(s.terms);
        }
    }
    if (w1 > 0.0)
        out.e1 = std::max(r1 / w1, 0.5);
    if (!r2.empty()) {
        std::vector<double> ones(r2.size(), 1.0);
        double a, b;
        if (lsq2(ones, g2, r2, w2, a, b)) {
            out.e2 = std::max(a, 0.5);
            out.g2 = std::max(b, 0.0);
        }
    }
    m = out;
    return true;
}

static double predicted_ms(phicomb_batch b) {
    t_model = b->model;
    double pred = 0.0;
    for (int g = 0; g < b->ng; ++g) {
        double t = 0.0;
        for (int it : b->sched.glist[g])
            t += cost_us(b->cost[it], b->sched.gsize[g]);
        pred = std::max(pred, t);
    }
    return pred * 1e-3;
}

// After a run: the measured duration of every instance (device clocks) and
// its measured term count refit the model; the schedule is rebuilt with it
// when that predicts a makespan 10 % below the run just measured.
void tune(phicomb_batch b, double measured_ms) {
    b->runs += 1;
    std::vector<Sample> smp;
    std::vector<int> group_of(b->count, 0);
    for (int g = 0; g < b->ng; ++g)
        for (int it : b->sched.glist[g])
            group_of[it] = g;
    for (int it = 0; it < b->count; ++it) {
        const int *info = b->info_host + 8 * it;
        const double terms = (double)std::max(1, info[1] + info[2]);
        b->cost[it].terms = terms;
        const double us =
            (double)(b->ts_host[2 * it + 1] - b->ts_host[2 * it]) / b->clock_khz * 1e3;
        if (!(us > 0.0))
            continue;
        const int G = b->sched.gsize[group_of[it]];
        smp.push_back({(double)G, rounds(b->cost[it], G), b->cost[it].cols, us / terms, terms});
    }
    b->last_measured_ms = measured_ms;
    b->last_predicted_ms = predicted_ms(b);   // this run's plan, term counts now measured
    Model m = b->model;
    if (fit_model(smp, m))
        b->model = m;
    b->refit_predicted_ms = predicted_ms(b);
    // keep the fastest plan measured so far; try a new one while the refit
    // predicts 10 % less than this run (at most kExplore times), and go back
    // to the best plan when a tried one measured slower
    if (!(b->best_ms > 0.0) || measured_ms < b->best_ms) {
        b->best_ms = measured_ms;
        b->best_sched = b->sched;
    }
    t_model = b->model;
    const Schedule trial = make_schedule(b->cost, b->cap);
    if (b->explored < kExplore && trial.makespan * 1e-3 < 0.9 * measured_ms) {
        b->explored += 1;
        build_plan(b, &trial);
    } else if (measured_ms > 1.02 * b->best_ms) {
        build_plan(b, &b->best_sched);
    }
}

}  // namespace

extern "C" {

int phicomb_batch_create(int count, const phicomb_batch_item *items, int precision,
                         phicomb_batch *out) {
    if (!out || !items || count < 1 || count > PHICOMB_MAX_BATCH)
        return PHICOMB_EINVAL;
    *out = nullptr;
    if (precision != PHICOMB_FP64 && precision != PHICOMB_MIXED)
        return PHICOMB_EINVAL;
    phicomb_batch b = new (std::nothrow) phicomb_batch_s();
    if (!b)
        return PHICOMB_ENOMEM;
    b->count = count;
    b->mix = (precision == PHICOMB_MIXED);
    int st = PHICOMB_OK;
    // validation and per-instance shapes
    for (int i = 0; i < count && st == PHICOMB_OK; ++i) {
        const phicomb_batch_item &q = items[i];
        if (!q.op || !q.prm || !q.t || !q.beta || !q.V || !q.W || q.p < 0 ||
            q.p > PHICOMB_MAX_P || q.r < 1 || q.r > PHICOMB_MAX_R || !(q.tol > 0.0) ||
            !std::isfinite(q.tol) || q.prm->status != PHICOMB_OK || !std::isfinite(q.prm->s) ||
            !std::isfinite(q.prm->shift) || q.prm->s < 0.0)
            st = PHICOMB_EINVAL;
        for (int k = 0; st == PHICOMB_OK && k < q.r; ++k)
            if (!std::isfinite(q.t[k]))
                st = PHICOMB_EINVAL;
        for (int k = 0; st == PHICOMB_OK && k < q.r * (q.p + 1); ++k)
            if (!std::isfinite(q.beta[k]))
                st = PHICOMB_EINVAL;
        if (st != PHICOMB_OK)
            break;
        // dense operators run through their CSR form in a batch
        const int kind = (q.op->dev.kind == kDense) ? kCsr : q.op->dev.kind;
        if (i == 0) {
            b->kind = kind;
            b->device = q.op->device;
        } else if (kind != b->kind || q.op->device != b->device) {
            st = PHICOMB_EINVAL;   // one operator kind and device per batch
        }
    }
    if (st == PHICOMB_OK && !(b->kernel = pick_batch_kernel(b->kind, b->mix)))
        st = PHICOMB_EINVAL;
    if (st != PHICOMB_OK) {
        free_batch(b);
        return st;
    }
    // workspace sizes and cost estimates
    std::vector<size_t> ws(count);
    b->cost.resize(count);
    size_t work_total = 0;
    b->ops.resize(count);
    b->p.resize(count);
    b->r.resize(count);
    b->s_int.resize(count);
    for (int i = 0; i < count; ++i) {
        const phicomb_batch_item &q = items[i];
        const int64_t n = q.op->dev.n;
        ws[i] = (solve_workspace_bytes(n, q.p, q.r, precision) + 255) & ~(size_t)255;
        work_total += ws[i];
        double tmax = 0.0;
        for (int k = 0; k < q.r; ++k)
            tmax = std::max(tmax, std::fabs(q.t[k]));
        const double sc = std::ceil(q.prm->s * tmax);
        if (!(sc <= 2147483647.0)) {
            free_batch(b);
            return PHICOMB_EINVAL;
        }
        const double steps = std::max(1.0, sc);
        const double k = taylor_terms(q.tol);
        b->cost[i].terms = k * steps;
        b->cost[i].cols = 2.0 * q.r;
        b->cost[i].n = n;
        b->cost[i].gmax = (int)std::max<int64_t>(1, std::min<int64_t>(256, (n + kNT - 1) / kNT));
        b->ops[i] = q.op;
        b->p[i] = q.p;
        b->r[i] = q.r;
    }
    b->cap = device_cus(b->device) / kXcds * kXcds;
    b->precision = precision;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->device) != hipSuccess ||
        khz <= 0)
        khz = 100000;
    b->clock_khz = (double)khz;
    // device memory: args | tables | info | clocks | work
    const size_t args_pad = (sizeof(SolveArgs) * count + 255) & ~(size_t)255;
    const size_t tab_b = (sizeof(int) * table_ints(count, b->cap) + 255) & ~(size_t)255;
    const size_t info_b = (sizeof(int) * 8 * count + 255) & ~(size_t)255;
    const size_t ts_b = (sizeof(long long) * 2 * count + 255) & ~(size_t)255;
    const size_t total = args_pad + tab_b + info_b + ts_b + work_total;
    if (hipSetDevice(b->device) != hipSuccess || hipMalloc(&b->mem, total) != hipSuccess ||
        hipHostMalloc((void **)&b->info_host, sizeof(int) * 8 * count, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void **)&b->ts_host, sizeof(long long) * 2 * count,
                      hipHostMallocDefault) != hipSuccess) {
        free_batch(b);
        return PHICOMB_ENOMEM;
    }
    char *base = (char *)b->mem;
    b->args = (SolveArgs *)base;
    b->tables = (int *)(base + args_pad);
    b->info_dev = (int *)(base + args_pad + tab_b);
    b->ts_dev = (long long *)(base + args_pad + tab_b + info_b);
    char *work = base + args_pad + tab_b + info_b + ts_b;
    std::vector<SolveArgs> args(count);
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        const phicomb_batch_item &q = items[i];
        st = build_solve_args(q.op, q.prm, q.p, q.r, q.t, q.beta, q.V, q.tol, precision, q.W,
                              work + off, ws[i], args[i]);
        if (st != PHICOMB_OK) {
            free_batch(b);
            return st;
        }
        off += ws[i];
        b->s_int[i] = args[i].s_int;
    }
    if (hipMemcpy(b->args, args.data(), sizeof(SolveArgs) * count, hipMemcpyHostToDevice) !=
        hipSuccess) {
        free_batch(b);
        return PHICOMB_EDEVICE;
    }
    st = build_plan(b);
    if (st == PHICOMB_OK &&
        hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
        st = PHICOMB_EDEVICE;
    if (st != PHICOMB_OK) {
        free_batch(b);
        return st;
    }
    *out = b;
    return PHICOMB_OK;
}

static hipError_t enqueue_batch(phicomb_batch b, hipStream_t s) {
    const int count = b->count, ng = b->ng;
    const int *t_variant = b->tables;
    const int *t_wg = t_variant + count;
    const int *t_gfirst = t_wg + b->wgs;
    const int *t_gsize = t_gfirst + ng;
    const int *t_goff = t_gsize + ng;
    const int *t_glist = t_goff + ng + 1;
    batch_sync_init<<<count, 256, 0, s>>>(b->args, count);
    const SolveArgs *a = b->args;
    long long *ts = b->ts_dev;
    void *kargs[] = {(void *)&a,       (void *)&t_variant, (void *)&t_wg,
                     (void *)&t_gfirst, (void *)&t_gsize,   (void *)&t_goff,
                     (void *)&t_glist,  (void *)&ts};
    hipError_t e = hipLaunchKernel((const void *)b->kernel, dim3(b->wgs), dim3(kNT), kargs, 0, s);
    if (e != hipSuccess)
        return e;
    batch_gather_info<<<(count * 8 + 255) / 256, 256, 0, s>>>(b->args, b->info_dev, count);
    e = hipMemcpyAsync(b->info_host, b->info_dev, sizeof(int) * 8 * count, hipMemcpyDeviceToHost,
                       s);
    if (e != hipSuccess)
        return e;
    return hipMemcpyAsync(b->ts_host, b->ts_dev, sizeof(long long) * 2 * count,
                          hipMemcpyDeviceToHost, s);
}

int phicomb_batch_run(phicomb_batch b, void *stream, phicomb_stats_t *stats) {
    if (!b)
        return PHICOMB_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
        return PHICOMB_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    // the launch is captured once per plan; a failed capture falls back to
    // direct launches
    if (!b->exec && !b->no_graph) {
        bool ok = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) ==
                  hipSuccess;
        if (ok) {
            const hipError_t e = enqueue_batch(b, b->cap_stream);
            hipGraph_t g = nullptr;
            ok = (hipStreamEndCapture(b->cap_stream, &g) == hipSuccess) && e == hipSuccess;
            if (ok && hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) == hipSuccess) {
                b->graph = g;
            } else {
                if (g)
                    hipGraphDestroy(g);
                b->exec = nullptr;
                hipGetLastError();
            }
        }
        if (!b->exec)
            b->no_graph = true;
    }
    const int held = round_xcd(b->wgs);
    if (cu_acquire(b->device, held, held) != held)
        return PHICOMB_EDEVICE;
    struct Hold {
        int dev, g;
        ~Hold() { cu_release(dev, g); }
    } hold{b->device, held};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timed = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    if (timed)
        hipEventRecord(e0, s);
    const hipError_t le = b->exec ? hipGraphLaunch(b->exec, s) : enqueue_batch(b, s);
    if (timed)
        hipEventRecord(e1, s);
    const bool synced = (le == hipSuccess) && hipStreamSynchronize(s) == hipSuccess;
    float ms = 0.0f;
    if (timed) {
        if (synced)
            hipEventElapsedTime(&ms, e0, e1);
        hipEventDestroy(e0);
        hipEventDestroy(e1);
    }
    if (!synced)
        return PHICOMB_EDEVICE;
    int worst = PHICOMB_OK;
    for (int i = 0; i < b->count; ++i) {
        const int *info = b->info_host + 8 * i;
        if (info[0] != PHICOMB_OK && worst == PHICOMB_OK)
            worst = info[0];
        if (stats) {
            phicomb_stats_t &o = stats[i];
            std::memset(&o, 0, sizeof(o));
            o.s_int = b->s_int[i];
            o.terms_S = info[1];
            o.terms_rec = info[2];
            o.max_terms_step = info[3];
            o.fp32_terms = info[4] + info[5];
            o.status = info[0];
            o.bytes_alg = solve_algorithmic_bytes(b->ops[i], b->p[i], b->r[i], b->s_int[i], info);
            o.ms = ms;
        }
    }
    if (worst == PHICOMB_OK)
        tune(b, ms);
    return worst;
}

int phicomb_batch_info(phicomb_batch b, int *groups, int *workgroups, double *predicted_ms) {
    if (!b)
        return PHICOMB_EINVAL;
    if (groups)
        *groups = b->ng;
    if (workgroups)
        *workgroups = b->wgs;
    if (predicted_ms)
        *predicted_ms = b->sched.makespan * 1e-3;
    return PHICOMB_OK;
}

int phicomb_batch_model(phicomb_batch b, double *get, const double *set) {
    if (!b)
        return PHICOMB_EINVAL;
    if (get) {
        get[0] = b->model.e1;
        get[1] = b->model.e2;
        get[2] = b->model.g2;
        get[3] = b->model.l0;
        get[4] = b->model.l1;
    }
    if (set) {
        for (int i = 0; i < 5; ++i)
            if (!(set[i] >= 0.0) || !std::isfinite(set[i]))
                return PHICOMB_EINVAL;
        b->model = Model{set[0], set[1], set[2], set[3], set[4]};
        return build_plan(b);
    }
    return PHICOMB_OK;
}

int phicomb_batch_fit(phicomb_batch b, double *measured_ms, double *predicted_ms_before,
                      double *predicted_ms_after) {
    if (!b)
        return PHICOMB_EINVAL;
    if (measured_ms)
        *measured_ms = b->last_measured_ms;
    if (predicted_ms_before)
        *predicted_ms_before = b->last_predicted_ms;
    if (predicted_ms_after)
        *predicted_ms_after = b->refit_predicted_ms;
    return PHICOMB_OK;
}

int phicomb_batch_times(phicomb_batch b, double *us, int *group_size) {
    if (!b)
        return PHICOMB_EINVAL;
    std::vector<int> group_of(b->count, 0);
    for (int g = 0; g < b->ng; ++g)
        for (int it : b->sched.glist[g])
            group_of[it] = g;
    for (int it = 0; it < b->count; ++it) {
        if (us)
            us[it] = (double)(b->ts_host[2 * it + 1] - b->ts_host[2 * it]) / b->clock_khz * 1e3;
        if (group_size)
            group_size[it] = b->sched.gsize[group_of[it]];
    }
    return PHICOMB_OK;
}

int phicomb_batch_destroy(phicomb_batch b) {
    if (!b)
        return PHICOMB_EINVAL;
    free_batch(b);
    return PHICOMB_OK;
}

}  // extern "C"
