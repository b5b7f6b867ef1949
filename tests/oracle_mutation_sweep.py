"""Mutation sweep over the oracle: how well do the CPU pins fix it?

Each mutant changes one site of one oracle module and reruns the oracle's
tests (tests/test_oracle_*.py) on a copy of the tree; a mutant that no test
fails is printed as a survivor.  Sites: + <-> -, * <-> /, < <-> <=, > <-> >=,
== <-> !=, a dropped unary minus, an integer constant plus one.

    python tests/oracle_mutation_sweep.py [module.py,...] [--workers N]

Not collected by pytest (a run takes minutes); it reads nothing but the
repository's own oracle/, inputs/ and tests/.
"""
from __future__ import annotations

import argparse
import ast
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import tempfile

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MODULES = ["aggregation.py", "amli.py", "cycle.py", "level.py", "poly.py", "spectral.py"]
SWAP = {ast.Add: ast.Sub, ast.Sub: ast.Add, ast.Mult: ast.Div, ast.Div: ast.Mult,
        ast.Lt: ast.LtE, ast.LtE: ast.Lt, ast.Gt: ast.GtE, ast.GtE: ast.Gt, ast.Eq: ast.NotEq, ast.NotEq: ast.Eq}


def _span(node):
    return (node.lineno, node.col_offset, node.end_lineno, node.end_col_offset)


def sites(tree):
    out = []
    for node in ast.walk(tree):
        if isinstance(node, ast.BinOp) and type(node.op) in SWAP:
            out.append(("binop", _span(node)))
        elif isinstance(node, ast.Compare) and len(node.ops) == 1 and type(node.ops[0]) in SWAP:
            out.append(("cmp", _span(node)))
        elif isinstance(node, ast.UnaryOp) and isinstance(node.op, ast.USub):
            out.append(("neg", _span(node)))
        elif isinstance(node, ast.Constant) and type(node.value) is int:
            out.append(("int", _span(node)))
    return out


class _Mutate(ast.NodeTransformer):
    def __init__(self, kind, span):
        self.kind, self.span = kind, span

    def _hit(self, node, kind):
        return self.kind == kind and _span(node) == self.span

    def visit_BinOp(self, node):
        self.generic_visit(node)
        if type(node.op) in SWAP and self._hit(node, "binop"):
            node.op = SWAP[type(node.op)]()
        return node

    def visit_Compare(self, node):
        self.generic_visit(node)
        if len(node.ops) == 1 and type(node.ops[0]) in SWAP and self._hit(node, "cmp"):
            node.ops = [SWAP[type(node.ops[0])]()]
        return node

    def visit_UnaryOp(self, node):
        self.generic_visit(node)
        if isinstance(node.op, ast.USub) and self._hit(node, "neg"):
            return node.operand
        return node

    def visit_Constant(self, node):
        if type(node.value) is int and self._hit(node, "int"):
            return ast.copy_location(ast.Constant(node.value + 1), node)
        return node


def _make_tree(root):
    os.makedirs(root)
    for d in ("oracle", "inputs", "tests"):
        shutil.copytree(os.path.join(REPO, d), os.path.join(root, d),
                        ignore=shutil.ignore_patterns("__pycache__"))
    shutil.copy(os.path.join(REPO, "pytest.ini"), root)


def _run_tests(root):
    env = dict(os.environ, OMP_NUM_THREADS="2", OPENBLAS_NUM_THREADS="2", MKL_NUM_THREADS="2")
    tests = sorted(t for t in os.listdir(os.path.join(root, "tests")) if t.startswith("test_oracle_"))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *[os.path.join("tests", t) for t in tests]],
                       cwd=root, env=env, capture_output=True, timeout=600)
    return r.returncode == 0


def _mutant(root, module, kind, span):
    path = os.path.join(REPO, "oracle", module)
    src = open(path).read()
    tree = _Mutate(kind, span).visit(ast.parse(src))
    ast.fix_missing_locations(tree)
    shutil.copy(path, os.path.join(root, "oracle", module + ".orig"))
    with open(os.path.join(root, "oracle", module), "w") as fh:
        fh.write(ast.unparse(tree))
    try:
        survived = _run_tests(root)
    finally:
        shutil.move(os.path.join(root, "oracle", module + ".orig"), os.path.join(root, "oracle", module))
    return survived, src.splitlines()[span[0] - 1].strip()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("modules", nargs="?", default=",".join(MODULES))
    ap.add_argument("--workers", type=int, default=4)
    a = ap.parse_args()
    jobs = []
    for module in a.modules.split(","):
        tree = ast.parse(open(os.path.join(REPO, "oracle", module)).read())
        jobs += [(module, kind, span) for kind, span in sites(tree)]
    print(f"{len(jobs)} mutants", flush=True)
    with tempfile.TemporaryDirectory() as tmp:
        roots = [os.path.join(tmp, f"w{i}") for i in range(a.workers)]
        for root in roots:
            _make_tree(root)
        if not _run_tests(roots[0]):
            sys.exit("the unmutated oracle fails its own tests")
        survivors = []
        free = list(roots)
        with cf.ThreadPoolExecutor(a.workers) as ex:
            pending, it = {}, iter(jobs)
            while True:
                for job in it:
                    root = free.pop()
                    pending[ex.submit(_mutant, root, *job)] = (root, job)
                    if not free:
                        break
                if not pending:
                    break
                done, _ = cf.wait(pending, return_when=cf.FIRST_COMPLETED)
                for fut in done:
                    root, (module, kind, span) = pending.pop(fut)
                    free.append(root)
                    survived, line = fut.result()
                    if survived:
                        survivors.append((module, span[0], kind, line))
                        print(f"SURVIVED {module}:{span[0]} {kind}: {line}", flush=True)
    print(f"{len(jobs) - len(survivors)} of {len(jobs)} mutants killed", flush=True)


if __name__ == "__main__":
    main()
