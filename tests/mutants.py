"""Planted errors in the oracle, on the CPU: a pin is only worth something if a
plausible mistake in the code it pins makes it fail.

``mutant(edits, workdir)`` copies the oracle's C sources into ``workdir``,
applies exact text replacements (each must match the stated number of times,
so a stale edit fails loudly instead of testing the unmodified oracle),
compiles the copy with the oracle's own flags and returns a second instance
of the ``oracle`` Python module bound to that library.
"""
import importlib.util
import itertools
import os
import shutil
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
_count = itertools.count()


def mutant(edits, workdir):
    """edits: list of (file, old, new) or (file, old, new, times)."""
    workdir = str(workdir)
    os.makedirs(workdir, exist_ok=True)
    for f in os.listdir(ORACLE):
        if f.endswith((".c", ".h")):
            shutil.copy(os.path.join(ORACLE, f), os.path.join(workdir, f))
    for e in edits:
        fname, old, new = e[:3]
        times = e[3] if len(e) > 3 else 1
        path = os.path.join(workdir, fname)
        with open(path) as fh:
            text = fh.read()
        assert text.count(old) == times, f"planted edit does not apply: {fname}: {old!r}"
        with open(path, "w") as fh:
            fh.write(text.replace(old, new))
    import oracle
    lib = os.path.join(workdir, "liborc_mutant.so")
    srcs = [os.path.join(workdir, s) for s in oracle._SOURCES]
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-w", "-o", lib] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    spec = importlib.util.spec_from_file_location(f"oracle_mutant_{next(_count)}",
                                                  os.path.join(ORACLE, "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod._LIB_PATH = lib
    mod._lib = None
    mod.lib()
    return mod


def fails(check, mod):
    """True if the pin ``check(mod)`` raises AssertionError on the mutant."""
    try:
        check(mod)
    except AssertionError:
        return True
    return False
