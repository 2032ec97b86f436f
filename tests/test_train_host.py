"""Host logic of the training module (no GPU): the pair filter and the
rough right-hand-side generator."""
import numpy as np
import torch

from paper_2503_00868_amd import train


def test_usable_pairs_drops_inconsistent_and_unresolved():
    rng = np.random.default_rng(0)
    n = 6
    e = rng.standard_normal((4, n, n, n))
    r = e.copy()                 # r.e > 0
    r[1] = -e[1]                 # r.e < 0: inconsistent pair
    r[2] = 1e-9 * e[2]           # residual far below the batch's largest
    r[3] = 0.5 * e[3]
    R = torch.tensor(r, dtype=torch.float32)
    E = torch.tensor(e, dtype=torch.float32)
    Rk, Ek, kept = train.usable_pairs(R, E)
    assert kept == 2
    assert torch.equal(Rk[0], R[0]) and torch.equal(Rk[1], R[3])
    assert torch.equal(Ek[1], E[3])


class _FaceSim:
    def __init__(self, n):
        self.n = n

    def to_faces(self, fields):
        return fields


def test_rough_field_is_seeded_localized_and_face_shaped():
    sim = _FaceSim(12)
    a = train.rough_field(sim, 5)
    b = train.rough_field(sim, 5)
    c = train.rough_field(sim, 6)
    assert [x.shape for x in a] == [(12, 12, 13), (12, 13, 12), (13, 12, 12)]
    assert all(np.array_equal(x, y) for x, y in zip(a, b))
    assert not all(np.array_equal(x, y) for x, y in zip(a, c))
    # the envelope makes it localized: most of the energy sits in a small part
    # of the box
    u = np.abs(a[0]).reshape(-1)
    top = np.sort(u)[::-1]
    assert top[: u.size // 4].sum() > 0.6 * u.sum()
