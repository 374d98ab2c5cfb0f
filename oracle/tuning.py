"""The searcher's outer loop, Alg. 1 (oracle; test infrastructure only),
Sect. 3.7, and the evaluation measure of Sect. 4.1.

Alg. 1 starts from a random configuration.  Each iteration profiles the
current configuration (runtime and counters), turns the counters into
required counter changes (the expert system, Sect. 3.5), scores every
configuration not evaluated yet with the model (Sect. 3.6), then runs
configurations drawn with score weights without profiling them; the fastest
of those becomes the next configuration to profile.  Every run, profiled or
not, is one empirical test.  The evaluation counts the empirical tests until
the first well-performing configuration (runtime within 1.1x of the best in
the space) is tested, averaged over many runs with different random numbers,
and compares it with random search.

Readings:
* draws per iteration: n, the number the text gives for runs without
  counters (n + 1 empirical tests per iteration, i (n + 1) in total; the
  listing's loop bound k <= n would draw n + 1); the default n is 5;
* "runs" are lookups in a table of measured runtimes and counters, as in the
  paper's simulated autotuning; a configuration profiled again (the fastest
  of the previous draws) is tested again;
* the next configuration to profile is the fastest drawn one, the later
  draw on a tie (t' <= t);
* random numbers: one 64-bit uniform per draw (the first draws the start);
* random search tests configurations in uniformly random order without
  repetition, so its expected number of tests to the first of K
  well-performing configurations among N is (N + 1) / (K + 1).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import expert as E
from . import search as SR


@dataclass
class Run:
    tested: list           # valid indices in test order
    profiled: list         # True for profiled runs
    tests_to_well: int     # 1-based position of the first well-performing test (0 if none)


def well_performing(runtime, factor: float = 1.1) -> np.ndarray:
    r = np.asarray(runtime, dtype=np.float64)
    return r <= factor * r.min()


def run(prep, runtime, counters, uniforms, draws: int = 5, max_tests: int = 1 << 30,
        cores: float = 1.0, threads: float = 1e9, reaction: float = 0.7,
        stop_at_well: bool = True) -> Run:
    """One run of Alg. 1 on table data.  ``prep`` carries the model's
    predictions (``prep.P32``) of every valid configuration."""
    runtime = np.asarray(runtime, dtype=np.float32)
    well = well_performing(runtime)
    explored = np.zeros(len(prep.valid), dtype=bool)
    C = prep.P32.shape[1]
    u = 0
    tested, profiled = [], []
    found = 0

    def test(l, prof):
        nonlocal found
        tested.append(int(l))
        profiled.append(prof)
        if not found and well[l]:
            found = len(tested)
        return (stop_at_well and found) or len(tested) >= max_tests

    r = SR.step(prep, explored, None, np.zeros(C, np.float32), [uniforms[u]], with_fp64=False)
    u += 1
    c = r.picks[0]
    while c is not None:
        if test(c, True):
            break
        _, _, d32, _ = E.expert_system(counters[c], False, cores, threads, reaction)
        picks = SR.step(prep, explored, c, d32[:C], uniforms[u:u + draws], with_fp64=False).picks
        u += draws
        best_t, nxt, stop = np.inf, None, False
        for l in picks:
            if l is None:
                break
            if test(l, False):
                stop = True
                break
            if runtime[l] <= best_t:
                best_t, nxt = runtime[l], l
        if stop:
            break
        c = nxt
    return Run(tested, profiled, found)


def random_search_expected(runtime) -> float:
    """Expected tests of random search to the first well-performing
    configuration: (N + 1) / (K + 1)."""
    well = well_performing(runtime)
    return (len(well) + 1) / (int(well.sum()) + 1)


def random_search(runtime, order) -> int:
    """Tests to the first well-performing configuration when testing in the
    given order (a permutation of the valid indices)."""
    well = well_performing(runtime)
    hits = np.flatnonzero(well[np.asarray(order)])
    return int(hits[0]) + 1 if len(hits) else 0
