"""CPU model of the device's batch protocol for iterative jobs (Fig. 2 on the
device), run under injected claim and completion orders.

The persistent kernel does not run Fig. 2 batch by batch.  Waves claim
trajectory indices below an issue limit, finished trajectories are added to
the counter word of the batch their index falls in, the wave whose addition
completes a batch evaluates it (eq. 4 on the estimate moved towards 0.5) and
publishes the next bound, and while a batch is pending the limit runs ahead
to the smallest bound any outcome of it could give.  This module restates
that protocol in Python (the same steps as the device code, one scheduler
action at a time) and checks, over many random schedules, that it ends with
Fig. 2's sequential result on the same verdicts: the same N, successes and
number of batches, with every index counted in its own batch.

Stale reads are modelled as the memory-ordering argument allows them: a
bound published before the issue limit passed a claimed index is visible to
the claiming wave; one published later may or may not be.  A negative
control drops that guarantee and must produce a miscount.
"""
import math
import random

import pytest

from oracle import wilson

DONE = 1 << 31
MAX_BATCHES = 32


def next_sample(p, eps, z, literal):
    return wilson.wilson_sample(wilson.rounded_estimate(p, eps, literal), eps, z)


class Job:
    def __init__(self, eps, z, literal=False, conservative=False):
        self.eps, self.z, self.literal = eps, z, literal
        self.capacity = wilson.wilson_sample(0.5, eps, z)
        n_first = wilson.wilson_sample(0.5 if conservative else 1.0, eps, z)
        self.bound = [0] * MAX_BATCHES
        self.pub_time = [math.inf] * MAX_BATCHES   # scheduler step of publication
        self.bound[0] = n_first
        self.pub_time[0] = -1
        self.cnt = [0] * MAX_BATCHES
        self.cnt[0] = DONE - n_first
        lim = n_first
        g = min(next_sample(0.0, eps, z, literal), next_sample(1.0, eps, z, literal))
        lim = max(lim, min(g, self.capacity))
        self.limit = lim
        self.next = 0
        self.cur = 0
        self.final = None
        self.error = False
        self.counted = {}        # index -> batch it was counted in

    def ns(self, p):
        return next_sample(p, self.eps, self.z, self.literal)


def evaluate(job, b, cw, now):
    """evaluate_batches: batch b is complete with counter word cw."""
    while True:
        Y = sum(job.cnt[q] >> 32 for q in range(b)) + (cw >> 32)
        Bb = job.bound[b]
        Np = job.ns(Y / Bb)
        if Np > Bb and Np < job.limit:
            job.error = True
            job.final = (Bb, Y, b + 1)
            return
        if Np > Bb and b + 1 < MAX_BATCHES and Np <= job.capacity:
            job.bound[b + 1] = Np
            job.pub_time[b + 1] = now
            job.cur = b + 1
            job.limit = max(job.limit, Np)
            flag = DONE - (Np - Bb)
            job.cnt[b + 1] += flag
            nw = job.cnt[b + 1]
            if (nw & 0xFFFFFFFF) == DONE:
                b, cw = b + 1, nw
                continue
            return
        job.final = (Bb, Y, b + 1)
        return


def speculate(job, c, cw):
    """speculate: raise the limit to the smallest next bound any outcome of
    pending batch c could give."""
    Bc = job.bound[c]
    Bp = job.bound[c - 1] if c else 0
    if Bc == 0:
        return
    size = Bc - Bp
    low = cw & 0xFFFFFFFF
    done = low + size - DONE if low + size >= DONE else low
    ylo = cw >> 32
    if done > size or ylo > done:
        return
    nlo = done - ylo
    yprev = sum(job.cnt[q] >> 32 for q in range(c))
    plo = (yprev + ylo) / Bc
    phi = (yprev + size - nlo) / Bc
    g = min(job.ns(plo), job.ns(phi))
    if job.literal and plo <= 0.5 <= phi:
        g = min(g, job.ns(0.5))
    if g > Bc:
        job.limit = max(job.limit, min(g, job.capacity))


def run_schedule(verdicts, job, rng, n_waves=4, ordered_visibility=True, group=True):
    """Drive one job to its end under a random schedule.  A wave holds its
    claimed indices (running on its lanes or waiting in its pool) until they
    finish; it claims again, as claim() does, once it holds fewer than a
    wave's worth.  Returns the number of scheduler steps taken."""
    flight = []          # (wave, index, claim step)
    held = [0] * n_waves
    step = 0
    while job.final is None:
        step += 1
        can_claim = [w for w in range(n_waves) if held[w] < 64 and job.next < job.limit]
        if not flight and not can_claim:
            raise AssertionError("stalled: nothing running and nothing claimable")
        if can_claim and (not flight or rng.random() < 0.35):
            w = rng.choice(can_claim)
            want = max((job.limit - job.next) // (4 * n_waves), 64 - held[w], 64)
            want = min(want, 256, job.limit - job.next)
            for i in range(job.next, job.next + want):
                flight.append((w, i, step))
            job.next += want
            held[w] += want
            continue
        # a random held trajectory finishes; with `group`, others of the same
        # wave finish in the same iteration and are added together
        k = rng.randrange(len(flight))
        w = flight[k][0]
        fin = [k]
        if group:
            fin += [q for q in range(len(flight)) if q != k and flight[q][0] == w and rng.random() < 0.1]
        done = [flight[q] for q in fin]
        for q in sorted(fin, reverse=True):
            flight.pop(q)
        held[w] -= len(done)
        # each lane's batch: the number of bounds at or below its index that it sees
        batches = []
        for (_, i, claimed) in done:
            b = 0
            for q in range(MAX_BATCHES - 1):
                bb = job.bound[q]
                visible = job.pub_time[q] <= claimed if ordered_visibility else job.pub_time[q] < 0
                if not visible and bb and rng.random() < 0.5:
                    visible = True
                if not visible:
                    bb = 0
                if bb == 0 or i < bb:
                    break
                b += 1
            batches.append(b)
        for b0 in sorted(set(batches)):
            sel = [i for (_, i, _), b in zip(done, batches) if b == b0]
            ny = sum(verdicts[i] for i in sel)
            for i in sel:
                job.counted[i] = b0
            old = job.cnt[b0]
            job.cnt[b0] += (ny << 32) | len(sel)
            nw = job.cnt[b0]
            if (nw & 0xFFFFFFFF) == DONE:
                evaluate(job, b0, nw, step)
            elif b0 == job.cur:
                if (old & 0xFFFFFFFF) == 0 or ((old >> 6) & 0x3FFFFFF) != ((nw >> 6) & 0x3FFFFFF):
                    speculate(job, b0, nw)
            if job.final is not None:
                break
    return step


def sequential(verdicts, eps, z, literal, conservative):
    def count_yes(lo, hi):
        return sum(verdicts[lo:hi])
    p_hat, lo, hi, n, yes, bounds = wilson.iterative_wilson(count_yes, eps, z, conservative, literal)
    return n, yes, len(bounds), bounds


CASES = [(p, eps, literal, conservative)
         for p in (0.0, 0.02, 0.3, 0.5, 0.8, 1.0)
         for eps in (0.05, 0.1)
         for literal in (False, True)
         for conservative in (False, True)
         if not (literal and conservative)]


@pytest.mark.parametrize("p,eps,literal,conservative", CASES)
def test_protocol_matches_fig2_under_random_schedules(p, eps, literal, conservative):
    z = wilson.z_value(0.95)
    for rep in range(6):
        rng = random.Random(hash((p, eps, literal, conservative, rep)) & 0xFFFFFFFF)
        cap = wilson.wilson_sample(0.5, eps, z)
        verdicts = [1 if rng.random() < p else 0 for _ in range(cap + 1)]
        n, yes, nb, bounds = sequential(verdicts, eps, z, literal, conservative)
        job = Job(eps, z, literal, conservative)
        run_schedule(verdicts, job, rng, n_waves=rng.choice((1, 2, 4, 8)))
        assert not job.error
        assert job.final == (n, yes, nb), (job.final, (n, yes, nb))
        # every index below N was counted, in the batch its index falls in
        lo = 0
        for b, hi in enumerate(bounds):
            for i in range(lo, hi):
                assert job.counted.get(i) == b, (i, job.counted.get(i), b)
            lo = hi


def test_unordered_bound_visibility_miscounts():
    """Negative control: if a claiming wave could miss a bound published
    before the limit passed its index, the protocol miscounts.  The ordering
    the device enforces (release before every raise of the limit, acquire on
    iterative claims) is what rules this out."""
    z = wilson.z_value(0.95)
    bad = 0
    for rep in range(40):
        rng = random.Random(1000 + rep)
        cap = wilson.wilson_sample(0.5, 0.05, z)
        verdicts = [1 if rng.random() < 0.3 else 0 for _ in range(cap + 1)]
        n, yes, nb, _ = sequential(verdicts, 0.05, z, False, False)
        job = Job(0.05, z)
        try:
            run_schedule(verdicts, job, rng, n_waves=2, ordered_visibility=False)
        except AssertionError:
            bad += 1
            continue
        if job.error or job.final != (n, yes, nb):
            bad += 1
    assert bad > 0
