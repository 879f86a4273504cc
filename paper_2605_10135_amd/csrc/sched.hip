// sched.hip -- host-side simulation of the shard-build task scheduler on
// cloud GPU instances, and the cost model (Sec. IV, "Cloud Instance Task
// Scheduler" and "Spot instance cost analysis").  No device code: it plans
// where the per-shard builds of the other files would run on a fleet of
// spot / on-demand instances and what that costs.
//
// The scheduler keeps a task list (pending shard builds) and an instance list
// (active, available, known remaining lifetime).  Availability-based policy:
// a task goes only to an idle active instance.  Time-based policy: only to an
// instance whose known remaining lifetime covers the task's estimated time
// (plus its data transfer); estimates are linear in shard size, fitted on
// sampled small builds.  A task whose instance terminates under it returns
// to the head of the task list and runs again (its partial work is lost).
// Events are taken from a min-heap; all events of one time are applied in a
// fixed order (terminations, then completions, by instance index) before one
// assignment pass over the idle instances in index order, so the schedule is
// deterministic.
#include <cmath>
#include <deque>
#include <limits>
#include <queue>
#include <vector>

#include "common.hpp"

namespace sg {
namespace sched {

struct Running {
    int task = -1;
    double start = 0.0, finish = 0.0;
};

}  // namespace sched
}  // namespace sg

using namespace sg;

extern "C" sg_status sg_cost_model(double overall_time, double gpu_active_time, double transfer_time,
                                   double cpu_price, double gpu_price, double* cost) {
    return guarded([&] {
        SG_REQUIRE(cost != nullptr, "cost is NULL");
        SG_REQUIRE(overall_time >= 0 && gpu_active_time >= 0 && transfer_time >= 0 && cpu_price >= 0 &&
                       gpu_price >= 0,
                   "times and prices must be >= 0");
        *cost = (overall_time + transfer_time) * cpu_price + (gpu_active_time + transfer_time) * gpu_price;
    });
}

extern "C" sg_status sg_sched_fit_linear(const double* sizes_h, const double* times_h, int32_t m, double* a,
                                         double* b) {
    return guarded([&] {
        SG_REQUIRE(m >= 1 && sizes_h != nullptr && times_h != nullptr && a != nullptr && b != nullptr,
                   "bad arguments");
        double sx = 0.0, sy = 0.0;
        for (int i = 0; i < m; ++i) {
            sx += sizes_h[i];
            sy += times_h[i];
        }
        const double mx = sx / m, my = sy / m;
        double sxx = 0.0, sxy = 0.0;
        for (int i = 0; i < m; ++i) {
            const double dx = sizes_h[i] - mx;
            sxx += dx * dx;
            sxy += dx * (times_h[i] - my);
        }
        *b = sxx > 0.0 ? sxy / sxx : 0.0;
        *a = my - *b * mx;
    });
}

extern "C" sg_status sg_sched_simulate(const double* est_h, const double* actual_h, int32_t T,
                                       const sg_instance* inst_h, int32_t G, int32_t time_based, double transfer,
                                       int32_t* task_instance_h, double* task_start_h, double* task_end_h,
                                       int32_t* attempts_h, double* summary_h) {
    return guarded([&] {
        SG_REQUIRE(T >= 0 && G >= 0, "T and G must be >= 0");
        SG_REQUIRE(T == 0 || (est_h != nullptr && actual_h != nullptr), "NULL task arrays");
        SG_REQUIRE(G == 0 || inst_h != nullptr, "NULL instance array");
        SG_REQUIRE(summary_h != nullptr, "summary is NULL");
        SG_REQUIRE(transfer >= 0 && std::isfinite(transfer), "transfer must be finite and >= 0");
        for (int i = 0; i < T; ++i)
            SG_REQUIRE(std::isfinite(est_h[i]) && std::isfinite(actual_h[i]) && est_h[i] >= 0 && actual_h[i] > 0,
                       "estimates must be finite >= 0 and actual times finite > 0");
        for (int g = 0; g < G; ++g)
            SG_REQUIRE(std::isfinite(inst_h[g].ready) && inst_h[g].ready >= 0 && inst_h[g].end > inst_h[g].ready &&
                           !std::isnan(inst_h[g].notice),
                       "instances need 0 <= ready < end (end may be +inf) and a notice time");
        constexpr double INF = std::numeric_limits<double>::infinity();

        std::deque<int> pending;
        for (int i = 0; i < T; ++i) pending.push_back(i);
        std::vector<sched::Running> run(G);
        std::vector<int32_t> inst(T, -1), att(T, 0);
        std::vector<double> t0(T, NAN), t1(T, NAN);
        double gpu_active = 0.0;
        int64_t preempt = 0;
        // event heap: every future time at which something may change
        std::priority_queue<double, std::vector<double>, std::greater<double>> ev;
        ev.push(0.0);
        for (int g = 0; g < G; ++g) {
            ev.push(inst_h[g].ready);
            if (inst_h[g].end != INF) ev.push(inst_h[g].end);
            if (inst_h[g].notice != INF && inst_h[g].notice > 0) ev.push(inst_h[g].notice);
        }
        int busy = 0;
        while (!ev.empty()) {
            const double now = ev.top();
            while (!ev.empty() && ev.top() == now) ev.pop();
            // terminations first: a task not finished by now is lost
            for (int g = 0; g < G; ++g) {
                if (inst_h[g].end == now && run[g].task >= 0 && run[g].finish > now) {
                    gpu_active += now - run[g].start;
                    ++preempt;
                    pending.push_front(run[g].task);
                    run[g].task = -1;
                    --busy;
                }
            }
            for (int g = 0; g < G; ++g) {
                if (run[g].task >= 0 && run[g].finish == now) {
                    const int k = run[g].task;
                    gpu_active += run[g].finish - run[g].start;
                    inst[k] = g;
                    t0[k] = run[g].start;
                    t1[k] = run[g].finish;
                    run[g].task = -1;
                    --busy;
                }
            }
            // one assignment pass over the idle active instances
            for (int g = 0; g < G && !pending.empty(); ++g) {
                const sg_instance& in = inst_h[g];
                if (run[g].task >= 0 || !(in.ready <= now && now < in.end)) continue;
                const bool known = time_based && in.notice <= now && in.end != INF;
                const double remaining = known ? in.end - now : INF;
                for (auto it = pending.begin(); it != pending.end(); ++it) {
                    if (transfer + est_h[*it] <= remaining) {
                        const int k = *it;
                        pending.erase(it);
                        ++att[k];
                        run[g].task = k;
                        run[g].start = now;
                        run[g].finish = now + transfer + actual_h[k];
                        ev.push(run[g].finish);
                        ++busy;
                        break;
                    }
                }
            }
            if (pending.empty() && busy == 0) break;
        }
        double makespan = 0.0;
        int32_t done = 0;
        for (int i = 0; i < T; ++i) {
            if (inst[i] >= 0) {
                makespan = std::max(makespan, t1[i]);
                ++done;
            }
            if (task_instance_h) task_instance_h[i] = inst[i];
            if (task_start_h) task_start_h[i] = t0[i];
            if (task_end_h) task_end_h[i] = t1[i];
            if (attempts_h) attempts_h[i] = att[i];
        }
        summary_h[0] = makespan;
        summary_h[1] = gpu_active;
        summary_h[2] = (double)preempt;
        summary_h[3] = (double)done;
    });
}
