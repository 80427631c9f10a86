"""Parser for the worked examples under tests/golden/ (plain text, one fact per line).

Line kinds:
  vars NAME=index ...                 variable names and their DIMACS numbers
  assignment NAME=T|F|U ...           one assignment per line, in slot order
  aggregate NAME=<letters> ...        expected aggregate assignment of all assignments
  clause LIT LIT ... | key=v[,v...]   a clause (-NAME for a negated literal) and the
                                      expected values, one per assignment in order
"""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
_VAL = {"T": 1, "F": -1, "U": 0}


def load(name):
    names, assignments, aggregate, clauses = {}, [], None, []
    with open(os.path.join(GOLDEN, name)) as fh:
        for raw in fh:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            kind, rest = line.split(None, 1)
            if kind == "vars":
                for tok in rest.split():
                    k, v = tok.split("=")
                    names[k] = int(v)
            elif kind == "assignment":
                a = {}
                for tok in rest.split():
                    k, v = tok.split("=")
                    a[names[k]] = _VAL[v]
                assignments.append(a)
            elif kind == "aggregate":
                aggregate = {}
                for tok in rest.split():
                    k, v = tok.split("=")
                    aggregate[names[k]] = frozenset(_VAL[ch] for ch in v)
            elif kind == "clause":
                body, exp = rest.split("|")
                lits = []
                for tok in body.split():
                    neg = tok.startswith("-")
                    v = names[tok.lstrip("-")]
                    lits.append(-v if neg else v)
                expect = {}
                for tok in exp.split():
                    k, v = tok.split("=")
                    expect[k] = [int(x) for x in v.split(",")]
                clauses.append((lits, expect))
            else:
                raise ValueError(f"{name}: unknown line kind {kind!r}")
    return dict(n_vars=max(names.values()), assignments=assignments, aggregate=aggregate, clauses=clauses)


def all_files():
    return sorted(f for f in os.listdir(GOLDEN) if f.endswith(".txt"))
