"""Free Join plans, written from the paper (oracle side; test infrastructure).

A plan is a list of nodes; a node is a list of subatoms ``(atom, vars)`` where
``atom`` is an atom index of the query and ``vars`` a tuple of variable ids in
the atom's column order (Section 3.2, definitions of subatom and plan).  The
first subatom of a node produced by ``binary2fj`` is the one it iterates.

Readings of the paper used here (each also listed in the design notes):

* binary2fj (Section 4.1, figure "bj2fj"): the "available" variables used
  when a relation is added to the current node are those of every node
  emitted so far *and* of the current node; with the narrower definition of
  Section 3.2 the worked examples of Section 4.1 do not come out.
* factor (Section 4.1, figure "factorize-plan"): the inner loop walks the
  node's lookups only (its subatoms after the first) and stops at the first
  that cannot move; walking the cover too would stop at once and contradict
  the worked clover example.  A moved lookup is appended to the previous
  node, after that node's own subatoms.
* Covers (Section 3.2): only *pure* covers, whose variables are exactly the
  node's new variables, are iterated; a plan whose node has none is refused.
* Schemas (Section 3.3 build phase): the list of an atom's subatom variable
  lists in plan order, with no extra trailing empty level; leaf multiplicities
  are supplied by the offset vectors instead.
"""

from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

Subatom = Tuple[int, Tuple[int, ...]]
Node = List[Subatom]
Plan = List[Node]


class PlanError(ValueError):
    pass


def atom_vars(query, a: int) -> Tuple[int, ...]:
    return tuple(query.atoms[a][1])


def binary2fj(query, order: Sequence[int]) -> Plan:
    """Left-deep binary plan [R1..Rm] (atom indices) -> Free Join plan
    (Section 4.1): node i covers the variables R_i adds to those of the
    relations before it and, for i < m, looks R_{i+1} up on the variables
    it shares with R_1..R_i."""
    order = list(order)
    if sorted(order) != list(range(len(query.atoms))):
        raise PlanError("the left-deep order must list every atom once")
    m = len(order)
    seen = [set()]                       # seen[i]: variables of R_1..R_i
    for a in order:
        seen.append(seen[-1] | set(atom_vars(query, a)))
    plan: Plan = []
    for i, a in enumerate(order):
        node = [(a, tuple(v for v in atom_vars(query, a) if v not in seen[i]))]
        if i + 1 < m:
            b = order[i + 1]
            node.append((b, tuple(v for v in atom_vars(query, b) if v in seen[i + 1])))
        plan.append(node)
    return plan


def node_vars(node: Node) -> set:
    out = set()
    for _, vs in node:
        out |= set(vs)
    return out


def avs(plan: Plan, k: int) -> set:
    """Variables of the nodes before node k."""
    out = set()
    for j in range(k):
        out |= node_vars(plan[j])
    return out


def factor(plan: Plan) -> Plan:
    """Conservative factoring: move lookups of node i to node i-1, from the
    last node backwards, while their variables are available before node i
    and node i-1 holds no subatom of the same atom."""
    plan = [list(node) for node in plan]
    n = len(plan)
    for i in range(n - 1, 0, -1):
        phi = plan[i]
        prev = plan[i - 1]
        before = avs(plan, i)
        moved = 0
        for alpha in list(phi[1:]):
            a, vs = alpha
            if set(vs) <= before and all(b != a for b, _ in prev):
                phi.remove(alpha)
                prev.append(alpha)
                moved += 1
            else:
                break
    return plan


def gj_plan(query, var_order: Sequence[int]) -> Plan:
    """Generic Join plan for a total variable order: node i holds A(v_i) for
    every atom A that contains v_i, in atom order (Section 3.2, eq. gj-plan)."""
    plan: Plan = []
    for v in var_order:
        node = [(a, (v,)) for a in range(len(query.atoms)) if v in atom_vars(query, a)]
        if not node:
            raise PlanError(f"variable {v} occurs in no atom")
        plan.append(node)
    return plan


def validate(query, plan: Plan) -> None:
    """Raise PlanError unless the plan partitions every atom and is valid
    (Section 3.2): (a) no atom twice in a node, (b) a cover exists."""
    if not plan:
        raise PlanError("empty plan")
    seen: Dict[int, List[int]] = {a: [] for a in range(len(query.atoms))}
    for node in plan:
        if not node:
            raise PlanError("empty node")
        atoms_here = [a for a, _ in node]
        if len(set(atoms_here)) != len(atoms_here):
            raise PlanError("validity (a): an atom occurs twice in one node")
        for a, vs in node:
            if a < 0 or a >= len(query.atoms):
                raise PlanError("unknown atom")
            if not set(vs) <= set(atom_vars(query, a)):
                raise PlanError("subatom variables are not the atom's")
            seen[a].extend(vs)
    for a in range(len(query.atoms)):
        if sorted(seen[a]) != sorted(atom_vars(query, a)):
            raise PlanError("the nodes do not partition an atom")
    for k, node in enumerate(plan):
        if not covers(plan, k):
            raise PlanError("validity (b): a node has no cover")


def covers(plan: Plan, k: int) -> List[int]:
    """Indices (within node k) of the subatoms containing all new variables."""
    new = node_vars(plan[k]) - avs(plan, k)
    return [i for i, (_, vs) in enumerate(plan[k]) if new <= set(vs)]


def pure_covers(plan: Plan, k: int) -> List[int]:
    """Covers that bind no variable already bound before node k."""
    before = avs(plan, k)
    return [i for i in covers(plan, k) if not (set(plan[k][i][1]) & before)]


def schemas(query, plan: Plan) -> List[List[Tuple[int, ...]]]:
    """Per atom, the variable lists of its subatoms in plan order."""
    out = [[] for _ in query.atoms]
    for node in plan:
        for a, vs in node:
            out[a].append(tuple(vs))
    return out


def plan_str(query, plan: Plan) -> str:
    """Render like the paper: [[R(x,a),S(x)],[S(b),T(x)],[T(c)]]."""
    names = query.var_names
    def rname(a):
        return getattr(query, "atom_names", None)[a] if getattr(query, "atom_names", None) else query.relations[query.atoms[a][0]].name
    parts = []
    for node in plan:
        parts.append("[" + ",".join(f"{rname(a)}({','.join(names[v] for v in vs)})" for a, vs in node) + "]")
    return "[" + ",".join(parts) + "]"


def root_is_built(query, plan: Plan, a: int) -> bool:
    """Build-phase rule: an atom's root map is built unless its first subatom
    is both the last level of its schema and the only pure cover of its
    node, in which case the base table (or its selection) is iterated as is
    (Section 4.2, iterating the base table directly)."""
    sch = schemas(query, plan)[a]
    for k, node in enumerate(plan):
        for i, (b, _) in enumerate(node):
            if b == a:
                pc = pure_covers(plan, k)
                return not (len(sch) == 1 and pc == [i])
    raise PlanError("atom not in plan")
