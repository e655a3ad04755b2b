"""Copies of the CPU reference with one planted mistake, for tests showing that a pin
catches it. A planted copy is the reference's source with a text substitution applied
(each old text must occur exactly once), compiled like the reference into a temporary
directory; `installed(lib)` makes the oracle module's wrappers call that copy."""
import contextlib
import ctypes
import os
import shutil
import tempfile

import oracle as O
from oracle.build import HERE, build_oracle

SOURCES = ("smc2_oracle.c", "smc2_oracle.h", "pf_real.inc", "mlp.inc")


def build_planted(name, edits, workdir=None):
    """edits: [(file, old, new)]. Returns the loaded library of the planted copy."""
    d = tempfile.mkdtemp(prefix="planted_%s_" % name, dir=workdir)
    for f in SOURCES:
        shutil.copy(os.path.join(HERE, f), d)
    for f, old, new in edits:
        p = os.path.join(d, f)
        text = open(p).read()
        assert text.count(old) == 1, "planted edit %r does not match %s exactly once" % (name, f)
        open(p, "w").write(text.replace(old, new))
    out = build_oracle(src_dir=d, out=os.path.join(d, "liboracle_planted.so"))
    lib = ctypes.CDLL(out)
    O._declare(lib)
    return lib


@contextlib.contextmanager
def installed(lib):
    """Route the oracle module's wrappers to `lib` inside the block."""
    saved = O.lib()
    O._lib = lib
    try:
        yield
    finally:
        O._lib = saved
