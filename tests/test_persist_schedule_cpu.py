"""CPU checks of the persistent batched kernel's task list (host only, no
device call): every task of every problem appears once, each task waits for
exactly the problem's tasks of its earlier passes, those tasks come earlier
in the list, and workgroups that take tasks in list order and wait as the
kernel does always finish, whatever their number and the tasks' durations
(a simulation of the kernel's protocol).  The simulation itself is checked
on a list with a dependency placed after its dependant, which it must
report as stuck."""
import os
import random

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1711_00005_amd", "libpe3d.so")


@pytest.fixture(scope="module")
def P():
    if not os.path.exists(LIB):
        pytest.fail("libpe3d.so is not built (run __graft_entry__.build())")
    import paper_1711_00005_amd.pe3d as _P
    return _P


def simulate(tasks, nprob, workers, durations):
    """Workgroups take tasks in list order; a task may start once its
    problem's finished-task count reaches `need`.  Returns the finish time
    of the last task, or None if the workers are stuck (every worker holds a
    task whose need can no longer be met)."""
    done = [0] * nprob
    nxt = 0
    running = []          # (finish time, problem) of started tasks
    waiting = []          # tasks taken but not started
    free = workers
    now = 0.0
    while nxt < len(tasks) or running or waiting:
        # workers take the next tasks in order
        while free > 0 and nxt < len(tasks):
            waiting.append(nxt)
            nxt += 1
            free -= 1
        started = True
        while started:
            started = False
            for t in list(waiting):
                p, need = tasks[t][0], tasks[t][5]
                if done[p] >= need:
                    waiting.remove(t)
                    running.append((now + durations[t], p))
                    started = True
        if not running:
            return None if waiting else now
        running.sort()
        now, p = running.pop(0)
        done[p] += 1
        free += 1
    return now


def shapes(seed):
    rng = random.Random(seed)
    n = rng.randint(1, 9)
    na = [rng.randint(1, 9) for _ in range(n)]
    asub = [rng.randint(1, 4) for _ in range(n)]
    nb = [rng.choice([0, rng.randint(1, 9)]) for _ in range(n)]
    nsub = [rng.randint(1, 4) for _ in range(n)]
    steps = [rng.randint(0, 5) for _ in range(n)]
    nch = rng.randint(1, 3)
    chain = [rng.randrange(nch) for _ in range(n)]
    # groups numbered from 0 within each chain
    group = []
    for i in range(n):
        group.append(rng.randint(0, 2))
    for c in range(nch):
        used = sorted({group[i] for i in range(n) if chain[i] == c})
        ren = {g: k for k, g in enumerate(used)}
        for i in range(n):
            if chain[i] == c:
                group[i] = ren[group[i]]
    return na, asub, nb, nsub, steps, chain, group


@pytest.mark.parametrize("seed", range(40))
def test_task_list_covers_every_tile_once_and_waits_for_earlier_passes(P, seed):
    na, asub, nb, nsub, steps, chain, group = shapes(seed)
    tasks = P.pe3d_persist_schedule(na, asub, nb, nsub, steps, chain, group)
    n = len(na)
    seen = {}
    for pos, (p, tile, k, kind, sub, need) in enumerate(tasks):
        assert 0 <= p < n and 0 <= k < steps[p]
        if kind == 0:
            assert sub == asub[p] and tile % asub[p] == 0 and 0 <= tile < na[p]
            key = [(p, k, 0, t) for t in range(tile, min(tile + sub, na[p]))]
        else:
            assert kind == 1 and nb[p] > 0 and sub == nsub[p]
            assert tile % nsub[p] == 0 and 0 <= tile < nb[p]
            key = [(p, k, 1, t) for t in range(tile, min(tile + sub, nb[p]))]
        for x in key:
            assert x not in seen, x
            seen[x] = pos
    expect = {(p, k, 0, t) for p in range(n) for k in range(steps[p]) for t in range(na[p])}
    expect |= {(p, k, 1, t) for p in range(n) for k in range(steps[p]) for t in range(nb[p])}
    assert set(seen) == expect
    # need = the problem's tasks of earlier passes (counted from the list, not
    # from a formula), and all of them precede the task
    for pos, (p, tile, k, kind, sub, need) in enumerate(tasks):
        earlier = [q for q, x in enumerate(tasks) if x[0] == p and (x[2], x[3]) < (k, kind)]
        assert need == len(earlier), (pos, tasks[pos])
        assert all(q < pos for q in earlier)


@pytest.mark.parametrize("seed", range(30))
def test_workers_taking_tasks_in_order_always_finish(P, seed):
    na, asub, nb, nsub, steps, chain, group = shapes(100 + seed)
    tasks = P.pe3d_persist_schedule(na, asub, nb, nsub, steps, chain, group)
    rng = random.Random(seed)
    for workers in (1, 2, 3, 8, 64):
        dur = [rng.uniform(0.1, 3.0) for _ in tasks]
        assert simulate(tasks, len(na), workers, dur) is not None, workers


def test_simulation_reports_a_dependency_placed_after_its_dependant(P):
    tasks = P.pe3d_persist_schedule([2], [1], [3], [1], [2], [0], [0])
    assert simulate(tasks, 1, 1, [1.0] * len(tasks)) is not None
    # the azimuth tasks of step 0 moved before the depth tasks they wait for
    bad = tasks[2:5] + tasks[0:2] + tasks[5:]
    assert simulate(bad, 1, 1, [1.0] * len(bad)) is None
    assert simulate(bad, 1, 3, [1.0] * len(bad)) is None


def test_phases_of_chains_are_interleaved(P):
    """Two chains of one problem each: the azimuth phase of chain 0's step 0
    comes after chain 1's depth phase of step 0 (the other chain's work
    covers the wait)."""
    tasks = P.pe3d_persist_schedule([2, 2], [1, 1], [2, 2], [1, 1], [2, 2], [0, 1], [0, 0])
    order = [(p, k, kind) for p, tile, k, kind, sub, need in tasks]
    first = {}
    for i, x in enumerate(order):
        first.setdefault(x, i)
    assert first[(0, 0, 0)] < first[(1, 0, 0)] < first[(0, 0, 1)] < first[(1, 0, 1)] < first[(0, 1, 0)]


def test_schedule_rejects_invalid_shapes(P):
    with pytest.raises(Exception):
        P.pe3d_persist_schedule([0], [1], [1], [1], [1], [0], [0])    # no depth tiles
    with pytest.raises(Exception):
        P.pe3d_persist_schedule([1], [1], [1], [17], [1], [0], [0])   # tiles per task above 16
    with pytest.raises(Exception):
        P.pe3d_persist_schedule([1], [0], [1], [1], [1], [0], [0])    # no depth tiles per task
    with pytest.raises(Exception):
        P.pe3d_persist_schedule([1], [1], [1], [1], [-1], [0], [0])   # negative steps


def test_batch_kernel_arguments_are_validated(P):
    with pytest.raises(Exception):
        P.pe3d_set_batch_kernel(2, 1.0)
    with pytest.raises(Exception):
        P.pe3d_set_batch_kernel(P.PE3D_BATCH_PERSISTENT, -1.0)
    with pytest.raises(Exception):
        P.pe3d_set_batch_kernel(P.PE3D_BATCH_PERSISTENT, float("nan"))
    with pytest.raises(Exception):
        P.pe3d_set_batch_kernel(P.PE3D_BATCH_PERSISTENT, 1e9)
    P.pe3d_set_batch_kernel(P.PE3D_BATCH_LAUNCHES, 1.0)
