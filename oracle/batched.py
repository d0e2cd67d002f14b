"""Independent environments, each solved by the float64 V-FPI oracle in turn
(the batched form runs the same per-environment algorithm side by side)."""
from __future__ import annotations

from .core import vfpi


def vfpi_envs(envs, **kw):
    """``envs``: list of per-environment problems.  Returns one result dict
    per environment (see ``core.vfpi``)."""
    return [vfpi(p, **kw) for p in envs]
