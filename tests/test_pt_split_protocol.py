"""Host model of the split PT form's energy mailbox (the protocol of
sg_pt_run_split, restated with Python threads): G groups of one run each
own T/G walkers; at step ti a group writes its walkers' words (tag ti + 1,
value) into half ti mod 2 of the run's [2][T] mailbox, then waits for the
other groups' words of the same tag.  Random delays between every action
explore the interleavings.  The model checks what the kernel relies on: a
reader never meets a later tag than the one it waits for (a word is never
overwritten before every group has read it), every value read is the value
written for that step, and every group sees the same energies each step.
A variant with a single-half mailbox (no double buffering) shows that the
check does catch the overwrite the second half prevents."""
import random
import threading
import time

import pytest


def _energy(step, w):
    return (step * 7919 + w * 104729) % 100003 - 50000


def _run(T, G, steps, halves, seed, slow0=0.0, wait_s=20.0):
    box = [[(0, 0) for _ in range(T)] for _ in range(halves)]   # (tag, value); zeroed first
    lock = threading.Lock()   # one word's 64-bit access is atomic in the kernel
    seen = [[None] * steps for _ in range(G)]
    errors = []
    TG = T // G

    def group(g):
        rng = random.Random(seed * 1000 + g)
        mine = range(g * TG, (g + 1) * TG)
        for ti in range(steps):
            tag = ti + 1
            half = ti % halves
            for w in mine:                          # publish
                if rng.random() < 0.3:
                    threading.Event().wait(rng.random() * 1e-4)
                with lock:
                    box[half][w] = (tag, _energy(ti, w))
            energies = {w: _energy(ti, w) for w in mine}
            if g == 0 and slow0:
                threading.Event().wait(slow0)   # group 0 lags between publishing and reading
            for w in range(T):                      # collect
                if w in mine:
                    continue
                deadline = time.monotonic() + wait_s
                while True:
                    with lock:
                        t_read, v = box[half][w]
                    if t_read == tag:
                        energies[w] = v
                        break
                    if t_read > tag:
                        errors.append(f"group {g} step {ti} walker {w}: tag {t_read} overwrote {tag}")
                        return
                    if time.monotonic() > deadline:
                        errors.append(f"group {g} step {ti} walker {w}: no word")
                        return
                    if rng.random() < 0.5:
                        threading.Event().wait(rng.random() * 1e-5)
            seen[g][ti] = tuple(energies[w] for w in range(T))
            if rng.random() < 0.2:                  # the sweep of the next step
                threading.Event().wait(rng.random() * 3e-4)

    threads = [threading.Thread(target=group, args=(g,)) for g in range(G)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    return seen, errors


@pytest.mark.parametrize("T,G,seed", [(8, 2, 1), (12, 4, 2), (16, 8, 3), (6, 2, 4)])
def test_double_buffered_mailbox_delivers_every_step(T, G, seed):
    steps = 60
    seen, errors = _run(T, G, steps, 2, seed)
    assert not errors, errors[:3]
    want = [tuple(_energy(ti, w) for w in range(T)) for ti in range(steps)]
    for g in range(G):
        assert seen[g] == want, g


def test_single_half_mailbox_is_caught_overwriting():
    # with one half the other groups publish step ti + 1 while group 0 has
    # not yet read step ti: the tag check sees the later tag
    _, errors = _run(8, 4, 6, 1, 100, slow0=0.05, wait_s=1.0)   # the others then wait in vain
    assert any(e.startswith("group 0") and "overwrote" in e for e in errors), errors[:3]
    # the same lag is harmless with the second half
    seen, errors = _run(8, 4, 6, 2, 100, slow0=0.05)
    assert not errors and all(seen[g] == seen[0] for g in range(4))
