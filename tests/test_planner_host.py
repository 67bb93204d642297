"""The batched SST* search (Sec. 5.2, Alg. 2) on the CPU with the oracle as its simulator:
it finds the passive design for a goal straight ahead, its pruning keeps the tree sparse
(no two active nodes within the radius where one costs no more than the other was
inserted after it), the radius follows the schedule of Alg. 2, and a given seed gives the
same tree."""
import math

import numpy as np

import oracle as O
from paper_2509_15180_amd import planner as PL
from paper_2509_15180_amd import workloads as W


def oracle_simulator(prob):
    def sim(designs, starts=None):  # every design from zero: starts are not used
        work = PL.design_instances(prob, designs)
        o = O.rollout(work, threads=4)
        n = work.inst_i[:, 0]
        idx = np.arange(len(n))
        st = np.where(np.arange(o["status"].shape[1])[None, :] < n[:, None], o["status"], 0).max(1)
        return o["tip"][idx, n - 1, :3], st, [o["theta"][q, :n[q]] for q in idx]
    return sim


def open_field(goal=(0.5, 0.0)):
    return PL.Problem(obstacles=np.zeros((0, 4)), kinds=np.zeros(0, np.int32), goal=goal,
                      goal_radius=0.05, max_links=40)


def test_straight_goal_is_reached_without_actuators():
    prob = open_field()
    pl = PL.BatchedSST(prob, oracle_simulator(prob), batch=16, seed=1)
    sol = pl.run(15)
    assert sol >= 0
    node = pl.nodes[sol]
    assert len(node.spams) == 0  # the cheapest design: no sPAM
    assert math.hypot(node.tip[0] - 0.5, node.tip[1]) <= 0.05
    acts = pl.path(sol)
    assert sum(a[0] for a in acts) + 1 == node.n and all(a[1] == 0 for a in acts)


def test_pruning_keeps_the_tree_sparse_and_the_schedule():
    """No two active nodes lie within the current radius (a node is inserted only when
    every active node within the radius costs more, and those are deactivated; nodes are
    never reactivated and the radius only shrinks)."""
    prob = PL.maze(0)
    prob.max_links = 40
    pl = PL.BatchedSST(prob, oracle_simulator(prob), batch=12, seed=2)
    radii = []
    for _ in range(9):
        pl.iterate()
        radii.append(pl.r)
        act = [k for k, nd in enumerate(pl.nodes) if nd.active]
        for a in act:
            for b in act:
                if a < b:
                    assert PL.se2_distance(pl.nodes[a].tip, pl.nodes[b].tip) > pl.r
    assert sum(not nd.active for nd in pl.nodes) > 0  # pruning deactivated some
    # r decays by alpha at iteration sst_iter0 = 7, the next update at
    # 7 + round(7 (1 + log2 2) 0.8^-(3 + 2 + 1) 2)
    assert radii[5] == 60.0 and abs(radii[6] - 48.0) < 1e-12
    assert pl.next_update == 7 + round(7 * 2 * 0.8 ** (-12))
    # costs: sPAM count plus length over the maximum length
    for nd in pl.nodes:
        assert nd.cost == len(nd.spams) + nd.n * prob.link_len / prob.max_length


def test_same_seed_same_tree():
    prob = PL.maze(1)
    prob.max_links = 30
    trees = []
    for _ in range(2):
        pl = PL.BatchedSST(prob, oracle_simulator(prob), batch=8, seed=5)
        for _ in range(3):
            pl.iterate()
        trees.append([(nd.parent, nd.n, nd.action, tuple(nd.tip)) for nd in pl.nodes])
    assert trees[0] == trees[1]


def test_se2_metric():
    assert PL.se2_distance((0, 0, 0), (0.06, 0, 0)) == 60.0
    assert abs(PL.se2_distance((0, 0, math.pi - 0.01), (0, 0, -math.pi + 0.01)) - math.degrees(0.02)) < 1e-9


def test_planner_designs_are_the_rollout_batch():
    """A design (n, sPAMs) becomes one robot with n links, the problem's body and
    environment and one sPAM row per actuated edge."""
    prob = PL.maze(0)
    work = PL.design_instances(prob, [(5, []), (12, [(0.1, 0.24, -1.0, 5000.0)])])
    assert isinstance(work, W.Workload) and work.n_inst == 2
    assert list(work.inst_i[:, 0]) == [5, 12]
    inst = work.instance(1)
    assert np.allclose(np.asarray(inst["spam"]).reshape(-1, 4), [(0.1, 0.24, -1.0, 5000.0)])
    assert len(inst["kind"]) == len(prob.kinds)


def _brute_prune(nodes, children, r):
    """The pruning rule written out over every pair: children cheapest first; a child is
    dropped when an active node within r costs no more, else inserted and the active
    nodes within r deactivated.  Returns the active flags and the inserted children."""
    nodes = [[tuple(t), c, a] for t, c, a in nodes]
    inserted = []
    for q in sorted(range(len(children)), key=lambda q: (children[q][1], q)):
        tip, cost = children[q]
        near = [nd for nd in nodes if nd[2] and PL.se2_distance(nd[0], tip) <= r]
        if any(nd[1] <= cost for nd in near):
            continue
        for nd in near:
            nd[2] = False
        nodes.append([tuple(tip), cost, True])
        inserted.append(q)
    return [nd[2] for nd in nodes], inserted


def test_pruning_equals_the_rule_over_every_pair():
    """The k-d tree search finds exactly the neighbours the rule names: random trees and
    children, with costs drawn from a few values (ties) and tips on a 10 mm lattice with
    headings 0 (distances exactly at the radius)."""
    rng = np.random.default_rng(11)
    prob = open_field()
    for trial in range(6):
        pl = PL.BatchedSST(prob, lambda d, s: (np.zeros((len(d), 3)), np.zeros(len(d), int),
                                                [np.zeros(n) for n, _ in d]), 8)
        pl.r = [60.0, 48.0, 38.4][trial % 3]
        lattice = trial % 2 == 0
        def tip():
            if lattice:
                return np.array([0.01 * rng.integers(0, 30), 0.01 * rng.integers(0, 30), 0.0])
            return np.array([rng.uniform(0, 0.3), rng.uniform(0, 0.3), rng.uniform(-3, 3)])
        for _ in range(120):  # an existing tree
            nd = PL.Node(parent=0, n=5, spams=[], action=(4, 0, 0.0), tip=tip(),
                         cost=float(rng.integers(0, 4)), active=bool(rng.random() < 0.7))
            pl._add(nd)
        before = [(nd.tip, nd.cost, nd.active) for nd in pl.nodes]
        children = [PL.Node(parent=0, n=5, spams=[], action=(4, 0, 0.0), tip=tip(),
                            cost=float(rng.integers(0, 4))) for _ in range(80)]
        want_active, want_ins = _brute_prune(before, [(c.tip, c.cost) for c in children], pl.r)
        m0 = len(pl.nodes)
        added = pl.prune_insert(children)
        assert [pl.nodes[k] for k in added] == [children[q] for q in want_ins]
        assert added == list(range(m0, m0 + len(added)))
        assert [nd.active for nd in pl.nodes] == want_active
        assert list(pl._active[:len(pl.nodes)]) == want_active


def _signed_distance(kind, o, x, y):
    """Distance from (x, y) to a circle (kind 0, radius o[2]) or an axis-aligned rectangle
    (kind 1, half sides o[2], o[3]); negative inside."""
    if kind == 0:
        return math.hypot(x - o[0], y - o[1]) - o[2]
    dx, dy = abs(x - o[0]) - o[2], abs(y - o[1]) - o[3]
    return math.hypot(max(dx, 0.0), max(dy, 0.0)) + min(max(dx, dy), 0.0)


def test_environments_start_clear_and_their_goals_are_free():
    """Every synthetic environment leaves the tube of the first links (base at the origin,
    heading +x) and the goal region free of obstacles, for several seeds."""
    for name, make in PL.ENVIRONMENTS.items():
        for seed in range(4):
            p = make(seed)
            base = min(_signed_distance(k, o, x, 0.0) for k, o in zip(p.kinds, p.obstacles)
                       for x in np.linspace(0.0, 0.1, 21))
            goal = min(_signed_distance(k, o, *p.goal) for k, o in zip(p.kinds, p.obstacles))
            assert base > p.tube_radius, (name, seed, base)
            assert goal > p.goal_radius, (name, seed, goal)
