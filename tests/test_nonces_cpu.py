"""Automatic nonces: one counter per key seed for the whole process, so that
no two reservations (engines, Pencil+ preprocessing, callers) share a Philox
stream (every random value is keyed by (seed, nonce))."""
import threading

import pytest

from paper_2403_11166_amd import api


def test_reservations_are_disjoint_and_per_seed():
    a = api.reserve_nonces(101, 5)
    b = api.reserve_nonces(101, 3)
    c = api.reserve_nonces(202, 1)
    assert a >= api.AUTO_NONCE_BASE and c >= api.AUTO_NONCE_BASE
    assert set(range(a, a + 5)).isdisjoint(range(b, b + 3))
    assert b == a + 5
    with pytest.raises(ValueError):
        api.reserve_nonces(101, 0)


def test_reservations_from_threads_never_overlap():
    got = []
    lock = threading.Lock()

    def worker():
        mine = [api.reserve_nonces(303, 2) for _ in range(200)]
        with lock:
            got.extend(mine)

    ths = [threading.Thread(target=worker) for _ in range(8)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    used = [n for first in got for n in (first, first + 1)]
    assert len(used) == len(set(used)) == 8 * 200 * 2


def test_fresh_seeds_differ():
    assert len({api.fresh_seed() for _ in range(16)}) == 16
