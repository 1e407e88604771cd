"""Small hand-made fixture graphs (out-edge CSR via graphgen.from_edges)."""
import numpy as np

import graphgen as gg


def cycle(n):
    u = np.arange(n)
    return gg.from_edges(n, u, (u + 1) % n, name=f"cycle{n}")


def complete(n):
    u, v = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = u != v
    return gg.from_edges(n, u[keep], v[keep], name=f"complete{n}")


def edgeless(n):
    return gg.from_edges(n, np.zeros(0), np.zeros(0), name=f"edgeless{n}")


def star_out(n):
    v = np.arange(1, n)
    return gg.from_edges(n, np.zeros(n - 1), v, name=f"star_out{n}")


def star_in(n):
    v = np.arange(1, n)
    return gg.from_edges(n, v, np.zeros(n - 1), name=f"star_in{n}")


def chain(n):
    u = np.arange(n - 1)
    return gg.from_edges(n, u, u + 1, name=f"chain{n}")


def dangling_mix():
    # 0->1, 0->2, 1->2, 2->0, 3->2 ; 4 dangling with an in-arc, 5 isolated
    src = [0, 0, 1, 2, 3, 1]
    dst = [1, 2, 2, 0, 2, 4]
    return gg.from_edges(6, src, dst, name="dangling_mix")


def two_components():
    src = [0, 1, 2, 3, 4, 5]
    dst = [1, 2, 0, 4, 5, 3]
    return gg.from_edges(6, src, dst, name="two_components")


def with_dups_and_loops():
    src = [0, 0, 0, 1, 1, 2, 2, 3]
    dst = [1, 1, 0, 2, 2, 2, 3, 0]
    return gg.from_edges(4, src, dst, name="dups_loops")


def random_small(n, m, seed):
    rng = np.random.default_rng(seed)
    return gg.from_edges(n, rng.integers(0, n, m), rng.integers(0, n, m), name=f"rand{n}_{m}_{seed}")


def all_small():
    return [cycle(7), complete(6), edgeless(5), star_out(9), star_in(9), chain(8), dangling_mix(),
            two_components(), with_dups_and_loops(), random_small(40, 120, 1), random_small(64, 64, 2),
            gg.rmat(6, 8, seed=3), gg.rmat(7, 4, seed=4)]
