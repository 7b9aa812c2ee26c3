"""Parse and print plans in the paper's notation, e.g. [[R(x,a),S(x)],[T(c)]].

Used by tests on queries whose atoms have distinct relation names."""

import re


def atom_index(query, name):
    hits = [a for a, (r, _) in enumerate(query.atoms) if query.relations[r].name == name]
    if len(hits) != 1:
        raise ValueError(f"relation name {name!r} is not unique in the query")
    return hits[0]


def parse_plan(query, text):
    text = text.replace(" ", "")
    if not (text.startswith("[[") and text.endswith("]]")):
        raise ValueError(text)
    nodes = []
    for node_txt in re.findall(r"\[([^\[\]]*)\]", text[1:-1]):
        node = []
        for name, vars_txt in re.findall(r"(\w+)\(([^()]*)\)", node_txt):
            vs = tuple(query.var_names.index(v) for v in vars_txt.split(",") if v)
            node.append((atom_index(query, name), vs))
        nodes.append(node)
    return nodes


def subatom_str(query, sub):
    a, vs = sub
    return f"{query.relations[query.atoms[a][0]].name}({','.join(query.var_names[v] for v in vs)})"


def plan_str(query, plan):
    return "[" + ",".join("[" + ",".join(subatom_str(query, s) for s in node) + "]" for node in plan) + "]"


def load_golden(path):
    rows = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([p.strip() for p in line.split("|")])
    return rows
