"""Class inheritance (Sec. 1.2: subclassing without wasted memory): a do-all
over a type visits that type and every type that inherits from it.  The
oracle's visit sets are pinned by hand-worked type lattices."""
import oracle


def test_types_without_parents_visit_only_themselves():
    parents = [None, None, None]
    for t in range(3):
        assert oracle.visit_types(parents, t) == {t}


def test_chain():
    # Animal <- Fish <- Shark: a do-all over Animal sees all three, over Fish
    # the fish and sharks, over Shark only sharks.
    parents = [None, 0, 1]
    assert oracle.visit_types(parents, 0) == {0, 1, 2}
    assert oracle.visit_types(parents, 1) == {1, 2}
    assert oracle.visit_types(parents, 2) == {2}


def test_tree_and_unrelated_type():
    #        0            4 (its own root)
    #      /   \\          |
    #     1     2          5
    #     |
    #     3
    parents = [None, 0, 0, 1, None, 4]
    assert oracle.visit_types(parents, 0) == {0, 1, 2, 3}
    assert oracle.visit_types(parents, 1) == {1, 3}
    assert oracle.visit_types(parents, 2) == {2}
    assert oracle.visit_types(parents, 3) == {3}
    assert oracle.visit_types(parents, 4) == {4, 5}
    assert oracle.visit_types(parents, 5) == {5}


def test_siblings_are_not_visited_through_each_other():
    parents = [None, 0, 0, 0]
    assert oracle.visit_types(parents, 2) == {2}
    assert oracle.visit_types(parents, 0) == {0, 1, 2, 3}


def test_deepest_chain_of_eight_types():
    parents = [None] + list(range(7))
    for t in range(8):
        assert oracle.visit_types(parents, t) == set(range(t, 8))


def test_parent_may_be_declared_after_its_child_in_the_model():
    # The model is only the inheritance relation; declaration order is a rule
    # of the heap description, not of the relation.
    parents = [2, None, None]
    assert oracle.visit_types(parents, 2) == {0, 2}


def test_cycles_and_bad_links_are_not_a_forest():
    assert oracle.visit_types([1, 0], 0) == set()
    assert oracle.visit_types([0], 0) == set()
    assert oracle.visit_types([None, 7], 0) == set()
