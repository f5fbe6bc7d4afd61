"""Class inheritance without wasted memory (Sec. 1.2): a subclass's blocks
hold only its own objects, in its own SOA layout, its first fields being the
parent's; a do-all over a type visits the type and every type inheriting
from it (the oracle's visit sets), reading the inherited fields by the
parent's field indices, and its deletes leave the subclasses' own fields
intact."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from paper_1809_07444_amd import _capi as C  # noqa: E402
from paper_1809_07444_amd.heap import Heap  # noqa: E402

# Shape {id, x}; Circle(Shape) {id, x, r}; Ring(Circle) {id, x, r, w: 8 bytes}; Label {id}.
TYPES = [(4, 4), (4, 4, 4), (4, 4, 4, 8), (4,)]
PARENTS = [None, 0, 1, None]
COUNTS = [3000, 2100, 1300, 900]


def build(capacity, width):
    heap = Heap(1024, capacity, TYPES, bitmap_width=width, parents=PARENTS)
    handles, ids = [], []
    nxt = 0
    for t, n in enumerate(COUNTS):
        h = heap.alloc_n(t, n)
        assert (h.cpu().numpy().view(np.uint32) != C.NULL).all()
        idv = torch.arange(nxt, nxt + n, dtype=torch.int32, device="cuda")
        heap.field_write(t, 0, h, idv)
        if t < 3:
            heap.field_write(t, 1, h, (idv.float() * 0.5).contiguous())
        if t in (1, 2):
            heap.field_write(t, 2, h, (idv * 7 + 1).contiguous())
        handles.append(h)
        ids.append(np.arange(nxt, nxt + n))
        nxt += n
    return heap, handles, ids, nxt


@pytest.mark.parametrize("capacity", [64, 0])
@pytest.mark.parametrize("width", [64, 32])
def test_do_all_visits_the_type_and_its_subclasses(capacity, width):
    heap, handles, ids, total = build(capacity, width)
    L = heap.layout()
    if capacity == 0:
        # Label (4 B) is the smallest type; each type has its own capacity.
        assert list(L.type_capacity[:4]) == [32, 16, 8, 64]
    for t in range(4):
        want = oracle.visit_types(PARENTS, t)
        counts = heap.visit_counts(t).cpu().numpy()
        for u in range(4):
            hu = handles[u].cpu().numpy().view(np.uint32)
            assert (counts[hu] == (1 if u in want else 0)).all(), (t, u)
        assert counts.sum() == sum(COUNTS[u] for u in want)
    # The heap counts each visit under the visited object's own type.
    st = heap.stats()
    assert st["visits"] == [COUNTS[u] * sum(u in oracle.visit_types(PARENTS, t) for t in range(4)) for u in range(4)]
    # The inherited field x, gathered by id through a do-all over Shape.
    x, present = heap.gather(0, 0, 1, total)
    pres = present.cpu().numpy().astype(bool)
    fam = np.concatenate(ids[:3])
    assert pres[fam].all() and pres.sum() == len(fam)
    assert np.array_equal(x.cpu().numpy().view(np.float32)[fam], fam.astype(np.float32) * 0.5)
    assert heap.check() == {}


@pytest.mark.parametrize("capacity", [64, 0])
def test_delete_through_the_parent_keeps_subclass_fields(capacity):
    heap, handles, ids, total = build(capacity, 64)
    heap.delete_if_mod(0, 0, 3, 0)          # every Shape, Circle and Ring with id % 3 == 0
    st = heap.stats()
    want = [int((i % 3 != 0).sum()) for i in ids[:3]] + [COUNTS[3]]
    assert st["live"][:4] == want
    assert st["frees"][:4] == [COUNTS[u] - want[u] for u in range(4)]
    # The survivors' own field r (past the inherited ones) is untouched.
    for u in (1, 2):
        keep = handles[u][torch.from_numpy(ids[u] % 3 != 0).cuda()]
        r = heap.field_read(u, 2, keep).cpu().numpy()
        assert np.array_equal(r, ids[u][ids[u] % 3 != 0] * 7 + 1)
    # A do-all over Circle now visits the surviving Circles and Rings only.
    counts = heap.visit_counts(1).cpu().numpy()
    assert counts.sum() == want[1] + want[2]
    assert heap.check() == {}
