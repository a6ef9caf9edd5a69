"""Host-thread model of the one-launch 2D sweep's ticket / flag protocol
(k_sweep2d in its queue form, run on the CPU; no GPU).

The items of a sweep are the (geometry, octant, chunk, 8 x 8 tile) work
items in the library's order: by tile diagonal of the octant's flow frame,
stable within a diagonal.  Item i waits for the items of its x- and y-upwind
tiles (same geometry, octant and chunk; none across the domain edge).  A
block of the launch, once running, takes the next ticket from a shared
counter and processes the item of that ticket; it waits (bounded number of
polls, giving up sets a shared abort word) for its upwind items, then
publishes its own.  The model runs the blocks as threads, at most `resident`
of them at a time, started in a random order, and shows:

* every upwind item precedes its dependent in the order (so a block waits
  only for tickets already taken, i.e. for blocks already running);
* with any number of resident blocks (one included) every item completes
  and nothing gives up;
* a dependency on a later item (a broken order) cannot hang the launch: the
  bounded wait gives up, the abort word is set and every block ends.
"""
import random
import threading

import pytest


def schedule(films, octants, nchunk):
    """Items (film, octant, chunk, tx, ty) in sweep order and their upwind
    item indices, built the way the library builds its 2D work list."""
    recs = []
    for f, (n0, n1) in enumerate(films):
        nt0, nt1 = (n0 + 7) // 8, (n1 + 7) // 8
        for o, (sg0, sg1) in enumerate(octants):
            for ty in range(nt1):
                for tx in range(nt0):
                    fx = tx if sg0 > 0 else nt0 - 1 - tx
                    fy = ty if sg1 > 0 else nt1 - 1 - ty
                    for ch in range(nchunk):
                        recs.append((fx + fy, (f, o, ch, tx, ty)))
    recs.sort(key=lambda r: r[0])   # stable, as std::stable_sort
    items = [r[1] for r in recs]
    at = {it: i for i, it in enumerate(items)}
    up = []
    for (f, o, ch, tx, ty) in items:
        n0, n1 = films[f]
        nt0, nt1 = (n0 + 7) // 8, (n1 + 7) // 8
        sg0, sg1 = octants[o]
        ux, uy = tx - sg0, ty - sg1
        upx = at[(f, o, ch, ux, ty)] if 0 <= ux < nt0 else -1
        upy = at[(f, o, ch, tx, uy)] if 0 <= uy < nt1 else -1
        up.append((upx, upy))
    return items, up


QUADRANTS = [(1, 1), (-1, 1), (-1, -1), (1, -1)]


def run_launch(up, resident, seed, spin=20000):
    """Blocks as threads: at most `resident` run at once (a block holds its
    slot from its start to its end), started in a random order."""
    n = len(up)
    lock = threading.Lock()
    state = {"ticket": 0, "abort": False}
    done = [False] * n
    order = []
    slots = threading.Semaphore(resident)

    def wait(u):
        for k in range(spin):
            if done[u]:
                return True
            if k % 64 == 63 and state["abort"]:
                return False
            threading.Event().wait(0)   # yield, like s_sleep
        state["abort"] = True
        return False

    def block():
        with slots:
            with lock:   # the ticket: an atomic add by the running block
                t = state["ticket"]
                state["ticket"] += 1
            ux, uy = up[t]
            if ux >= 0:
                wait(ux)
            if uy >= 0:
                wait(uy)
            with lock:
                order.append(t)
            done[t] = True   # publish after the block's stores

    threads = [threading.Thread(target=block) for _ in range(n)]
    random.Random(seed).shuffle(threads)
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=60)
        assert not th.is_alive(), "a block did not end"
    return done, state["abort"], order


def test_upwind_items_precede_their_dependents():
    films = [(16, 24), (40, 8), (8, 8), (33, 17)]
    items, up = schedule(films, QUADRANTS, 3)
    assert len(items) == len(set(items))
    for i, (ux, uy) in enumerate(up):
        assert ux < i and uy < i
    # every item but the first tile of each (geometry, octant, chunk) waits
    n_first = len(films) * len(QUADRANTS) * 3
    assert sum(1 for ux, uy in up if ux < 0 and uy < 0) == n_first


@pytest.mark.parametrize("resident", [1, 3, 16])
@pytest.mark.parametrize("seed", [0, 1])
def test_every_item_completes_for_any_residency(resident, seed):
    _, up = schedule([(24, 16), (16, 32)], QUADRANTS, 2)
    done, aborted, order = run_launch(up, resident, seed)
    assert all(done) and not aborted
    # a block published only after its upwind items
    pos = {t: k for k, t in enumerate(order)}
    for i, (ux, uy) in enumerate(up):
        for u in (ux, uy):
            if u >= 0:
                assert pos[u] < pos[i]


def test_a_broken_order_gives_up_instead_of_hanging():
    _, up = schedule([(16, 16)], QUADRANTS[:1], 1)
    up = list(up)
    up[0] = (len(up) - 1, -1)   # the first ticket waits for the last item
    done, aborted, _ = run_launch(up, 1, 0, spin=2000)
    assert aborted              # the bounded wait gave up and every block ended
