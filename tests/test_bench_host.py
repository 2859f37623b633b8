"""Host-side logic of bench.py, without a GPU: the algorithmic byte counts
behind the roofline figures, and the single-GPU guard."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_algorithmic_bytes_of_the_gmres_iteration():
    """200x200x50 cells, 13.88M blocks: the apply reads every off-diagonal
    block and D^-1 once plus four block vectors (7.62 GB); the fused lower
    half of the SpMV adds the lower blocks and four vectors (3.55 GB):
    about 5,586 bytes per cell in all, halved in FP32 storage."""
    b = bench.algorithmic_bytes(2_000_000, 13_880_000)
    assert b["ilu_apply"] == 7_618_560_000
    assert b["ilu_spmv"] == 11_171_840_000
    assert round(b["ilu_spmv"] / 2_000_000) == 5_586
    assert b["ilu_spmv32"] == b["ilu_spmv"] // 2
    assert b["spmv"] == (13_880_000 - 2_000_000) * 512 + 2 * 2_000_000 * 64


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr


def _unbound_names(path):
    """Names a function of the module reads that nothing binds: not its
    parameters or locals (nor an enclosing function's), not a module-level
    name, not a builtin -- what would raise NameError only when the benchmark
    reaches that line on the GPU."""
    import ast
    import builtins
    tree = ast.parse(open(path).read())
    module = set(dir(builtins)) | {"__file__", "__name__", "__doc__", "__spec__", "__package__"}
    for node in tree.body:
        if isinstance(node, (ast.FunctionDef, ast.ClassDef)):
            module.add(node.name)
        elif isinstance(node, (ast.Import, ast.ImportFrom)):
            module.update((a.asname or a.name).split(".")[0] for a in node.names)
        elif isinstance(node, (ast.Assign, ast.AnnAssign)):
            for t in (node.targets if isinstance(node, ast.Assign) else [node.target]):
                module.update(n.id for n in ast.walk(t) if isinstance(n, ast.Name))

    def bound_in(fn):
        names = {a.arg for a in ast.walk(fn.args) if isinstance(a, ast.arg)}
        for n in ast.walk(fn):
            if isinstance(n, ast.Name) and isinstance(n.ctx, (ast.Store, ast.Del)):
                names.add(n.id)
            elif isinstance(n, (ast.Import, ast.ImportFrom)):
                names.update((a.asname or a.name).split(".")[0] for a in n.names)
            elif isinstance(n, (ast.FunctionDef, ast.Lambda)) and n is not fn:
                names.update(a.arg for a in ast.walk(n.args) if isinstance(a, ast.arg))
                if isinstance(n, ast.FunctionDef):
                    names.add(n.name)
            elif isinstance(n, ast.ExceptHandler) and n.name:
                names.add(n.name)
            elif isinstance(n, ast.comprehension):
                names.update(x.id for x in ast.walk(n.target) if isinstance(x, ast.Name))
        return names

    missing = []
    for fn in (n for n in ast.walk(tree) if isinstance(n, ast.FunctionDef)):
        ok = module | bound_in(fn)
        for outer in (n for n in ast.walk(tree) if isinstance(n, ast.FunctionDef) and n is not fn):
            if any(x is fn for x in ast.walk(outer)):
                ok |= bound_in(outer)
        for n in ast.walk(fn):
            if isinstance(n, ast.Name) and isinstance(n.ctx, ast.Load) and n.id not in ok:
                missing.append((fn.name, n.id, n.lineno))
    return missing


def test_every_name_the_benchmark_reads_is_bound():
    assert _unbound_names(os.path.join(ROOT, "bench.py")) == []


def test_driver_counts_solving_iterations_and_cuts_failed_steps():
    """bench.Driver on a scripted context (CPU tensors): a converged call ends
    the time step without counting; an update counts; an attempt that runs
    past max_newton or fails is restored and its step halved."""
    import types

    import torch

    import bench
    from paper_1811_11992_amd import isc

    class Scripted:
        def __init__(self, script):
            self.script, self.k = list(script), 0

        def isc_newton_step(self, u, u_old, dt, tol, lin):
            what = self.script[self.k]
            self.k += 1
            info = types.SimpleNamespace(converged=int(what == "c"),
                                         lin=types.SimpleNamespace(iters=5, inner_iters_total=0))
            if what == "u":
                u += 1.0
            return (isc.ISC_OK if what != "e" else isc.ISC_ERR_NEWTON_NOCONV), info

    d = bench.Driver.__new__(bench.Driver)
    d.ctx = Scripted("uuc" + "uuu" + "u" + "e" + "u")
    d.wl = types.SimpleNamespace(dt=8.0)
    d.lin, d.tol, d.max_newton = None, 1e-10, 2
    d.u = torch.zeros(3, dtype=torch.float64)
    d.u_old = d.u.clone()
    d.dt = 8.0
    d.ni_in_step = d.ni = d.lin_its = d.inner_its = d.steps_done = d.cuts = 0
    d.lin_each = []
    for _ in range(2):                 # two updates of the first step
        d.newton_iteration()
    assert (d.ni, d.steps_done, float(d.u[0])) == (2, 0, 2.0)
    d.newton_iteration()               # converged: next step, then its first update
    assert (d.ni, d.steps_done, float(d.u_old[0]), float(d.u[0])) == (3, 1, 2.0, 3.0)
    d.newton_iteration()               # second update of step 2
    d.newton_iteration()               # third call runs past max_newton: cut, then an update at dt/2
    assert (d.ni, d.cuts, d.dt, float(d.u[0])) == (5, 1, 4.0, 3.0)
    d.newton_iteration()               # an error: cut again, then an update at dt/4
    assert (d.ni, d.cuts, d.dt, float(d.u[0])) == (6, 2, 2.0, 3.0)
    assert d.lin_each == [5] * 6
