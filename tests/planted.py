"""Copies of the CPU oracle with one planted mistake, for showing that a pin
catches that mistake.  Only the tests use this; it edits the oracle's C
source in a temporary directory and never touches the real build."""
from __future__ import annotations

import contextlib
import os
import subprocess

from oracle import build as oracle_build
from oracle import oracle as O

SRC = os.path.join(oracle_build.HERE, "oracle.c")


def _function_span(src: str, head: str):
    a = src.index(head)
    b = src.index("\n}\n", a) + 3
    return a, b


def mutant_source(head: str, old: str, new: str) -> str:
    """oracle.c with `old` replaced by `new` inside the function whose
    definition starts with `head`; `old` must occur there exactly once."""
    src = open(SRC).read()
    a, b = _function_span(src, head)
    body = src[a:b]
    assert body.count(old) == 1, f"{old!r} occurs {body.count(old)} times in {head!r}"
    return src[:a] + body.replace(old, new) + src[b:]


@contextlib.contextmanager
def planted(tmpdir, head: str, old: str, new: str):
    """Binds the oracle wrapper to a build with the mistake for the duration
    of the block."""
    tag = str(abs(hash((head, old, new))))
    c_path = os.path.join(str(tmpdir), f"oracle_{tag}.c")
    so_path = os.path.join(str(tmpdir), f"liboracle_{tag}.so")
    with open(c_path, "w") as f:
        f.write(mutant_source(head, old, new))
    subprocess.run(["gcc", *oracle_build.CFLAGS, "-I", oracle_build.HERE, "-o", so_path, c_path,
                    "-lm"], check=True, capture_output=True)
    prev = O.use_library(so_path)
    try:
        yield O
    finally:
        O.use_library(prev)
