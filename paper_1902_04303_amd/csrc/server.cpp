// Serving form: a request loop over one context with keys resident on the device.
//
// Jobs (encrypted GWAS inputs) are submitted at any time.  A worker thread admits queued jobs while
// their device footprint fits the budget (and a cap on jobs in flight), then iterates: the fixed parts
// of newly admitted jobs run together (one batch per shape), and chunks of SNP batches are drawn from
// all active jobs of a shape, so work of jobs that arrived while others were on the GPU overlaps with
// theirs (continuous batching at chunk granularity).  A job completes when its last SNP batch is done;
// its latency is completion minus submission.  Results do not depend on the mix: every operation acts
// ciphertext by ciphertext.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>

#include "gwas.h"

namespace gck {

size_t input_footprint(const ckks_ctx &c, const EncInput &in) {
    auto bytes = [](const Ct &p) { return p ? p->data.words * 8 : 0; };
    size_t b = bytes(in.y) + bytes(in.S) + bytes(in.Xrep) + bytes(in.S_rep);
    for (auto &p : in.x) b += bytes(p);
    for (auto &p : in.A) b += bytes(p);
    // outputs, the fixed-part values kept for the per-batch part, and working space of the fixed part
    const size_t limb = (size_t)c.p.n * 8;
    const int nb = in.S ? in.S->count : 0, k = in.lay.k;
    b += (size_t)nb * 2 * (3 + 2 + 1 + 1) * limb;
    b += (size_t)k * 2 * (6 + 4) * limb + 2 * 2 * 3 * limb;
    b += (size_t)(k + 1) * 2 * (c.p.levels + 1) * limb * 4;
    return b;
}

}  // namespace gck

using namespace gck;
using Clock = std::chrono::steady_clock;

struct gwas_server {
    ckks_ctx *ctx = nullptr;
    size_t budget = 0;
    int max_jobs = 0, chunk = 0;

    struct Job {
        uint64_t id = 0;
        std::unique_ptr<gwas_enc_input> in;
        std::unique_ptr<gwas_enc_output> out;
        FixedOut fx;
        size_t footprint = 0;
        int remaining = 0;
        int state = 0;   // 0 queued, 1 admitted (fixed part pending), 2 active, 3 done, 4 cancelled
        bool counted = false;   // footprint included in in_flight_bytes (from admission until released)
        Clock::time_point t_submit, t_done;
    };

    std::mutex m;
    std::condition_variable cv, done_cv;
    std::deque<Job *> queue;
    std::vector<Job *> active;
    std::deque<std::pair<Job *, int>> work;   // pending (job, SNP batch) items, FIFO
    std::map<uint64_t, std::unique_ptr<Job>> jobs;
    uint64_t next_id = 1;
    size_t in_flight_bytes = 0;
    bool stop = false;
    bool sweep = false;   // an admitted or active job was cancelled: the worker releases its resources
    std::thread worker;
    std::string error;
    // statistics
    std::vector<double> latencies_ms;
    Clock::time_point first_submit, last_done;
    bool any = false;
    int peak_in_flight = 0;
    uint64_t iterations = 0;

    // Free what a finished or cancelled job holds on the device (its input and the fixed-part values) and
    // return its footprint to the budget, once.  Called by the worker with m and the context lock held.
    void release(Job *j) {
        j->fx = FixedOut{};
        j->in.reset();
        if (j->counted) {
            in_flight_bytes -= j->footprint;
            j->counted = false;
        }
    }

    void run() {
        for (;;) {
            std::vector<Job *> admitted;
            {
                std::unique_lock<std::mutex> lk(m);
                cv.wait(lk, [&] { return stop || sweep || !queue.empty() || !work.empty(); });
                if (stop) return;
                while (!queue.empty() && (int)active.size() + (int)admitted.size() < max_jobs) {
                    Job *j = queue.front();
                    if (j->state == 4) { queue.pop_front(); continue; }
                    const bool fits = in_flight_bytes + j->footprint <= budget;
                    if (!fits && !(active.empty() && admitted.empty())) break;   // wait for memory
                    queue.pop_front();
                    in_flight_bytes += j->footprint;
                    j->counted = true;
                    j->state = 1;
                    admitted.push_back(j);
                }
                peak_in_flight = std::max(peak_in_flight, (int)(active.size() + admitted.size()));
            }
            try {
                std::lock_guard<std::recursive_mutex> ck(ctx->mu);
                if (!admitted.empty()) {
                    std::map<std::tuple<int, int, int, int>, std::vector<Job *>> buckets;
                    for (Job *j : admitted) buckets[bucket_of(*j->in->in)].push_back(j);
                    for (auto &kv : buckets) {
                        std::vector<const EncInput *> ins;
                        for (Job *j : kv.second) ins.push_back(j->in->in.get());
                        std::vector<FixedOut> fxs;
                        std::vector<EncOutput> reps;
                        fixed_for_jobs(*ctx, ins, fxs, reps);
                        std::lock_guard<std::mutex> lk(m);
                        for (size_t q = 0; q < kv.second.size(); ++q) {
                            Job *j = kv.second[q];
                            if (j->state == 4) {   // cancelled while its fixed part ran: nothing is queued
                                release(j);
                                continue;
                            }
                            j->fx = std::move(fxs[q]);
                            j->out = std::make_unique<gwas_enc_output>();
                            j->out->ctx = ctx;
                            j->out->lay = j->in->in->lay;
                            j->out->out = std::move(reps[q]);
                            j->remaining = j->in->in->S->count;
                            j->state = 2;
                            active.push_back(j);
                            for (int b = 0; b < j->remaining; ++b) work.push_back({j, b});
                        }
                    }
                }
                // one chunk of SNP batches of the shape of the oldest pending item
                std::vector<WorkItem> items;
                std::vector<Job *> owners;
                {
                    std::lock_guard<std::mutex> lk(m);
                    while (!work.empty() && work.front().first->state == 4) work.pop_front();
                    if (!work.empty()) {
                        auto shape = bucket_of(*work.front().first->in->in);
                        for (auto it = work.begin(); it != work.end() && (int)items.size() < chunk;) {
                            Job *j = it->first;
                            if (j->state == 4) { it = work.erase(it); continue; }
                            if (bucket_of(*j->in->in) == shape) {
                                items.push_back(WorkItem{j->in->in.get(), &j->fx, &j->out->out, it->second});
                                owners.push_back(j);
                                it = work.erase(it);
                            } else {
                                ++it;
                            }
                        }
                    }
                }
                if (!items.empty()) chunk_for_jobs(*ctx, items);
                GCK_HIP(hipStreamSynchronize(ctx->stream));
                ++iterations;
                std::lock_guard<std::mutex> lk(m);
                const auto now = Clock::now();
                for (Job *j : owners) {
                    if (--j->remaining == 0 && j->state == 2) {
                        j->state = 3;
                        j->t_done = now;
                        last_done = now;
                        latencies_ms.push_back(std::chrono::duration<double, std::milli>(now - j->t_submit).count());
                        release(j);
                        active.erase(std::find(active.begin(), active.end(), j));
                    }
                }
                // cancelled active jobs: no chunk references them any more (the chunk above has finished)
                for (auto it = active.begin(); it != active.end();) {
                    if ((*it)->state == 4) {
                        release(*it);
                        (*it)->out.reset();
                        it = active.erase(it);
                    } else {
                        ++it;
                    }
                }
                sweep = false;
                done_cv.notify_all();
            } catch (const std::exception &e) {
                std::lock_guard<std::mutex> lk(m);
                error = e.what();
                stop = true;
                done_cv.notify_all();
                return;
            }
        }
    }
};

namespace gck {
void set_last_error(const std::string &s);
}

namespace {
template <typename F>
int sguard(F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return CKKS_E_INVALID_ARG;
    }
}
}  // namespace

extern "C" {

int gwas_server_create(ckks_ctx *ctx, size_t hbm_budget_bytes, int max_jobs_in_flight, int chunk, gwas_server **out) {
    return sguard([&] {
        if (!ctx || !out || max_jobs_in_flight < 1 || chunk < 1) throw Error(CKKS_E_INVALID_ARG, "bad arguments");
        auto s = std::make_unique<gwas_server>();
        s->ctx = ctx;
        s->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)-1;
        s->max_jobs = max_jobs_in_flight;
        s->chunk = chunk;
        gwas_server *p = s.get();
        s->worker = std::thread([p] { p->run(); });
        *out = s.release();
        return CKKS_OK;
    });
}

void gwas_server_destroy(gwas_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->m);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    delete s;
}

int gwas_input_footprint(const gwas_enc_input *in, size_t *bytes) {
    return sguard([&] {
        if (!in || !bytes) throw Error(CKKS_E_INVALID_ARG, "null argument");
        *bytes = input_footprint(*in->ctx, *in->in);
        return CKKS_OK;
    });
}

int gwas_server_submit(gwas_server *s, gwas_enc_input *in, uint64_t *job_id) {
    return sguard([&] {
        if (!s || !in || !job_id) throw Error(CKKS_E_INVALID_ARG, "null argument");
        if (in->ctx != s->ctx) throw Error(CKKS_E_PARAM_MISMATCH, "input belongs to another context");
        {
            std::lock_guard<std::mutex> lk(s->m);
            if (!s->error.empty()) throw Error(CKKS_E_HIP, "server stopped: " + s->error);
        }
        size_t fp = input_footprint(*s->ctx, *in->in);
        if (fp > s->budget) {   // larger than the whole budget: keep its SNP batches on the host
            std::lock_guard<std::recursive_mutex> ck(s->ctx->mu);
            spill_snp(*s->ctx, *in->in);   // on failure the input is unchanged and still the caller's
            fp = input_footprint(*s->ctx, *in->in);
        }
        auto j = std::make_unique<gwas_server::Job>();
        j->footprint = fp;
        j->t_submit = Clock::now();
        std::lock_guard<std::mutex> lk(s->m);
        if (!s->error.empty()) throw Error(CKKS_E_HIP, "server stopped: " + s->error);
        // nothing below throws: ownership of the input passes to the server only on success
        j->in.reset(in);
        j->id = s->next_id++;
        *job_id = j->id;
        if (!s->any) {
            s->first_submit = j->t_submit;
            s->any = true;
        }
        s->queue.push_back(j.get());
        s->jobs[j->id] = std::move(j);
        s->cv.notify_all();
        return CKKS_OK;
    });
}

int gwas_server_poll(gwas_server *s, uint64_t job_id, int wait, gwas_enc_output **out) {
    return sguard([&] {
        if (!s || !out) throw Error(CKKS_E_INVALID_ARG, "null argument");
        std::unique_lock<std::mutex> lk(s->m);
        auto it = s->jobs.find(job_id);
        if (it == s->jobs.end()) throw Error(CKKS_E_INVALID_ARG, "unknown job");
        gwas_server::Job *j = it->second.get();
        if (wait) s->done_cv.wait(lk, [&] { return j->state >= 3 || !s->error.empty(); });
        if (!s->error.empty() && j->state < 3) throw Error(CKKS_E_HIP, "server stopped: " + s->error);
        if (j->state == 4) return (int)CKKS_E_CANCELLED;
        if (j->state != 3) return (int)CKKS_E_NOT_READY;
        *out = j->out.release();
        s->jobs.erase(it);
        return (int)CKKS_OK;
    });
}

int gwas_server_cancel(gwas_server *s, uint64_t job_id) {
    return sguard([&] {
        if (!s) throw Error(CKKS_E_INVALID_ARG, "null server");
        std::lock_guard<std::mutex> lk(s->m);
        auto it = s->jobs.find(job_id);
        if (it == s->jobs.end()) throw Error(CKKS_E_INVALID_ARG, "unknown job");
        gwas_server::Job *j = it->second.get();
        if (j->state == 3 || j->state == 4) return (int)CKKS_OK;
        // A queued job holds no budget and is skipped at admission.  An admitted or active job may be in
        // the worker's hands right now: the worker releases its memory and budget once no launch reads it.
        if (j->state == 1 || j->state == 2) s->sweep = true;
        j->state = 4;
        s->cv.notify_all();
        s->done_cv.notify_all();
        return (int)CKKS_OK;
    });
}

int gwas_server_stats(gwas_server *s, double *p50_ms, double *p99_ms, double *jobs_per_s, uint64_t *completed,
                      int *peak_jobs_in_flight) {
    return sguard([&] {
        if (!s) throw Error(CKKS_E_INVALID_ARG, "null server");
        std::lock_guard<std::mutex> lk(s->m);
        std::vector<double> v = s->latencies_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) {
            if (v.empty()) return 0.0;
            size_t i = (size_t)std::ceil(p * v.size()) - 1;
            return v[std::min(i, v.size() - 1)];
        };
        if (p50_ms) *p50_ms = pct(0.50);
        if (p99_ms) *p99_ms = pct(0.99);
        if (completed) *completed = v.size();
        if (jobs_per_s) {
            double span = s->any && !v.empty()
                              ? std::chrono::duration<double>(s->last_done - s->first_submit).count()
                              : 0.0;
            *jobs_per_s = span > 0 ? v.size() / span : 0.0;
        }
        if (peak_jobs_in_flight) *peak_jobs_in_flight = s->peak_in_flight;
        return CKKS_OK;
    });
}

}  // extern "C"
