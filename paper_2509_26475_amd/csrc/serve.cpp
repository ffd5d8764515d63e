// Request serving with continuous batching: requests are admitted in arrival
// order as soon as their device footprint fits the memory budget and a slot
// is free; admitted solves run at the same time on their own streams, each
// with a share of the CUs from the device's workgroup-slot ledger; results
// are collected by polling.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <new>
#include <thread>

#include "internal.h"

using namespace phc;

struct phicomb_req_s {
    phicomb_op op;
    phicomb_params_t prm;
    int p, r, precision;
    double t[PHICOMB_MAX_R];
    double beta[PHICOMB_MAX_R * (PHICOMB_MAX_P + 1)];
    const void *V;
    void *W;
    double tol;
    int64_t bytes;
    std::atomic<int> state{0};   // 0 queued, 1 running, 2 done
    int status = PHICOMB_PENDING;
    phicomb_stats_t stats{};
};

namespace {

struct Worker {
    hipStream_t stream = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    double *pinned = nullptr;
};

// One per process, never destroyed: its worker threads wait on its
// condition variable until the process ends.
class Server {
  public:
    static Server &get() {
        static Server *s = new Server();
        return *s;
    }

    int configure(int64_t budget, int slots) {
        std::lock_guard<std::mutex> g(mu_);
        if (budget > 0)
            budget_ = budget;
        if (slots > 0) {
            if ((int)workers_ > slots)
                return PHICOMB_EINVAL;   // slots can grow, not shrink
            slots_ = slots;
        }
        return PHICOMB_OK;
    }

    int submit(phicomb_req req) {
        std::unique_lock<std::mutex> g(mu_);
        if (req->bytes > budget_)
            return PHICOMB_EADMIT;
        while (workers_ < slots_) {
            ++workers_;
            std::thread([this]() { run(); }).detach();
        }
        queue_.push_back(req);
        cv_.notify_all();
        return PHICOMB_OK;
    }

  private:
    Server() {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0)
            budget_ = (int64_t)(free_b / 2);
        else
            budget_ = (int64_t)1 << 33;
        device_ = 0;
        hipGetDevice(&device_);
    }

    // First request in arrival order whose footprint fits the free budget:
    // a large request waiting for memory does not hold back smaller ones.
    phicomb_req take_locked() {
        for (auto it = queue_.begin(); it != queue_.end(); ++it) {
            if (in_use_ + (*it)->bytes <= budget_) {
                phicomb_req q = *it;
                queue_.erase(it);
                in_use_ += q->bytes;
                return q;
            }
        }
        return nullptr;
    }

    void run() {
        Worker w;
        hipSetDevice(device_);
        const bool ok =
            hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking) == hipSuccess &&
            hipHostMalloc((void **)&w.pinned, 64 * sizeof(double), hipHostMallocDefault) ==
                hipSuccess;
        for (;;) {
            phicomb_req q = nullptr;
            int floor_g = 1;
            {
                std::unique_lock<std::mutex> g(mu_);
                cv_.wait(g, [&]() { return (q = take_locked()) != nullptr; });
                // every running solve is guaranteed a 1/slots share of the CUs
                floor_g = std::max(1, device_cus(device_) / std::max(1, slots_));
            }
            q->state.store(1);
            int st = ok ? PHICOMB_OK : PHICOMB_EDEVICE;
            const size_t need = solve_workspace_bytes(q->op->dev.n, q->p, q->r, q->precision,
                                                      op_lr_rank(q->op));
            if (st == PHICOMB_OK && w.ws_bytes < need) {
                if (w.ws)
                    hipFree(w.ws);
                w.ws = nullptr;
                w.ws_bytes = 0;
                if (hipMalloc(&w.ws, need) != hipSuccess)
                    st = PHICOMB_ENOMEM;
                else
                    w.ws_bytes = need;
            }
            if (st == PHICOMB_OK)
                st = solve_run(q->op, &q->prm, q->p, q->r, q->t, q->beta, q->V, q->tol,
                               q->precision, q->W, w.stream, &q->stats, w.ws, w.ws_bytes,
                               w.pinned, floor_g);
            q->stats.status = st;
            q->status = st;
            {
                std::lock_guard<std::mutex> g(mu_);
                in_use_ -= q->bytes;
            }
            q->state.store(2);
            cv_.notify_all();
        }
    }

    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<phicomb_req> queue_;
    int workers_ = 0;
    int64_t budget_ = 0, in_use_ = 0;
    int slots_ = 4;
    int device_ = 0;
};

bool finite_array(const double *a, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i]))
            return false;
    return true;
}

}  // namespace

extern "C" {

int64_t phicomb_request_bytes(int64_t n, int p, int r, int precision) {
    if (n < 1 || p < 0 || r < 1)
        return -1;
    return (int64_t)solve_workspace_bytes(n, p, r, precision) + 8 * n * (p + 1 + r);
}

int phicomb_serve_config(int64_t budget_bytes, int slots) {
    if (slots > 64)
        return PHICOMB_EINVAL;
    return Server::get().configure(budget_bytes, slots);
}

int phicomb_submit(phicomb_op op, const phicomb_params_t *prm, int p, int r, const double *t,
                   const double *beta, const void *V, double tol, int precision, void *W,
                   phicomb_req *out) {
    if (!op || !prm || !t || !beta || !V || !W || !out)
        return PHICOMB_EINVAL;
    if (p < 0 || p > PHICOMB_MAX_P || r < 1 || r > PHICOMB_MAX_R)
        return PHICOMB_EINVAL;
    if (!(tol > 0.0) || !std::isfinite(tol) || prm->status != PHICOMB_OK)
        return PHICOMB_EINVAL;
    if (!std::isfinite(prm->shift) || !std::isfinite(prm->s) || prm->s < 0.0)
        return PHICOMB_EINVAL;
    if (!finite_array(t, r) || !finite_array(beta, (int64_t)r * (p + 1)))
        return PHICOMB_EINVAL;
    if (precision != PHICOMB_FP64 && precision != PHICOMB_MIXED)
        return PHICOMB_EINVAL;
    double tmax = 0.0;
    for (int i = 0; i < r; ++i)
        tmax = std::max(tmax, std::fabs(t[i]));
    if (!(std::ceil(prm->s * tmax) <= 2147483647.0))
        return PHICOMB_EINVAL;
    phicomb_req q = new (std::nothrow) phicomb_req_s();
    if (!q)
        return PHICOMB_ENOMEM;
    q->op = op;
    q->prm = *prm;
    q->p = p;
    q->r = r;
    q->precision = precision;
    std::memcpy(q->t, t, sizeof(double) * r);
    std::memcpy(q->beta, beta, sizeof(double) * r * (p + 1));
    q->V = V;
    q->W = W;
    q->tol = tol;
    q->bytes = (int64_t)solve_workspace_bytes(op->dev.n, p, r, precision, op_lr_rank(op)) +
               8 * op->dev.n * (p + 1 + r);
    const int st = Server::get().submit(q);
    if (st != PHICOMB_OK) {
        delete q;
        return st;
    }
    *out = q;
    return PHICOMB_OK;
}

int phicomb_poll(phicomb_req req, phicomb_stats_t *stats) {
    if (!req)
        return PHICOMB_EINVAL;
    if (req->state.load() != 2)
        return PHICOMB_PENDING;
    const int st = req->status;
    if (stats)
        *stats = req->stats;
    delete req;
    return st;
}

}  // extern "C"
