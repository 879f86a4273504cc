"""Plain reference of the spot-instance task scheduler and the cost model.

TEST INFRASTRUCTURE ONLY (like the rest of this package): the tests use it to
check the library's scheduler simulation; the product path never imports it.

Follows Sec. IV, "Cloud Instance Task Scheduler": a task list of pending
shard-build tasks and an instance list whose entries are active (rented and
not terminated), available (not running a task) and, when known, carry their
remaining lifetime; tasks go only to available instances (availability-based
policy) and, with the time-based policy, only to instances whose known
remaining lifetime covers the task's estimated time; a task whose instance is
terminated under it goes back to the task list and runs again elsewhere.
Estimated times are linear in shard size (fitted on sampled small builds).
And Sec. IV, "Spot instance cost analysis": cost = (overall time + transfer
time) x CPU price + (aggregated GPU active time + transfer time) x GPU price.

Readings where the paper is silent (the same ones the library takes):
  * time advances by events; at one time, terminations are handled first (a
    task whose finish time equals the termination time completes), then
    completions, then instances that become active, then one assignment pass
    over the idle active instances in index order;
  * an instance picks the first task in the task list whose estimate (plus the
    per-task transfer time) fits its known remaining lifetime (all tasks fit
    one whose lifetime is unknown, and every instance when the time-based
    policy is off); with none, it stays idle;
  * a preempted task returns to the head of the task list (the scheduler
    reallocates it first) and its partial work is lost;
  * the lifetime of an instance becomes known at its notice time (a notice at
    or before activation models a guaranteed duration);
  * a task occupies its instance for transfer + actual time; the GPU active
    time is the sum of every occupation, lost work included.
Written as a plain loop over event times, no priority queue.
"""
from __future__ import annotations

import math


def cost(overall_time, gpu_active_time, transfer_time, cpu_price, gpu_price):
    """The cost formula of Sec. IV (spot instance cost analysis)."""
    return (overall_time + transfer_time) * cpu_price + (gpu_active_time + transfer_time) * gpu_price


def fit_linear(sizes, times):
    """Least-squares line time = a + b * size through sampled builds (Sec. IV,
    time-based scheduling: build time scales linearly with shard size)."""
    n = len(sizes)
    mx = sum(sizes) / n
    my = sum(times) / n
    sxx = sum((x - mx) * (x - mx) for x in sizes)
    sxy = sum((x - mx) * (y - my) for x, y in zip(sizes, times))
    b = sxy / sxx if sxx > 0 else 0.0
    return my - b * mx, b


def simulate(est, actual, instances, time_based=True, transfer=0.0):
    """instances: list of dicts with keys ready, end, notice (math.inf allowed).
    Returns dict: task_instance, task_start, task_end, attempts (per task),
    makespan, gpu_active, preemptions, log (list of (task, instance, start,
    stop, completed))."""
    T, G = len(est), len(instances)
    pending = list(range(T))
    running = [None] * G          # (task, start, finish) or None
    done_inst = [-1] * T
    t_start = [math.nan] * T
    t_end = [math.nan] * T
    attempts = [0] * T
    log = []
    gpu_active = 0.0
    preemptions = 0
    now = -math.inf

    def alive(g, t):
        return instances[g]["ready"] <= t < instances[g]["end"]

    while True:
        # the next event time after `now`
        cands = []
        for g, ins in enumerate(instances):
            for key in ("ready", "end", "notice"):
                v = ins[key]
                if v > now and v != math.inf:
                    cands.append(v)
            if running[g] is not None and running[g][2] > now:
                cands.append(running[g][2])
        if now == -math.inf:
            cands.append(0.0)
        if not cands:
            break
        now = min(cands)
        # 1. terminations: a running task that has not finished by now is lost
        for g, ins in enumerate(instances):
            if ins["end"] == now and running[g] is not None:
                task, start, finish = running[g]
                if finish > now:
                    log.append((task, g, start, now, False))
                    gpu_active += now - start
                    preemptions += 1
                    pending.insert(0, task)
                    running[g] = None
        # 2. completions
        for g in range(G):
            if running[g] is not None and running[g][2] == now:
                task, start, finish = running[g]
                log.append((task, g, start, finish, True))
                gpu_active += finish - start
                done_inst[task] = g
                t_start[task] = start
                t_end[task] = finish
                running[g] = None
        # 3./4. one assignment pass over idle active instances, in index order
        for g, ins in enumerate(instances):
            if running[g] is not None or not alive(g, now) or not pending:
                continue
            known = time_based and ins["notice"] <= now and ins["end"] != math.inf
            remaining = ins["end"] - now if known else math.inf
            for i, task in enumerate(pending):
                if transfer + est[task] <= remaining:
                    pending.pop(i)
                    attempts[task] += 1
                    running[g] = (task, now, now + transfer + actual[task])
                    break
        if not pending and all(r is None for r in running):
            break
    makespan = max((e for e in t_end if not math.isnan(e)), default=0.0)
    return dict(task_instance=done_inst, task_start=t_start, task_end=t_end, attempts=attempts,
                makespan=makespan, gpu_active=gpu_active, preemptions=preemptions, log=log)
