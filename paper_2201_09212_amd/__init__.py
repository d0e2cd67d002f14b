"""V-FPI contact solver for AMD Instinct MI355X (gfx950).

The solver itself is the HIP library ``libvfpi.so`` (C ABI in
``include/vfpi.h``).  This package is its binding: ``_abi`` mirrors the C entry
points under the same names, ``solver`` wraps them for torch device tensors,
``autograd`` puts the adjoint behind ``torch.autograd.Function``, ``autotune``
picks launch variants.  Importing the package does not load the library; the
first call does, and raises if it has not been built.
"""
from ._abi import (VfpiError, load, vfpi_create, vfpi_destroy, vfpi_error_string, vfpi_step, vfpi_step_backward,
                   vfpi_timing_enable, vfpi_timing_read, vfpi_vnode_pattern, vfpi_vnode_values,
                   vfpi_step_batched, vfpi_tape_bytes)
from .solver import (Bsr, Contacts, Solver, bsr_from_arrays, contacts_from_arrays, make_opts, new_stats, read_stats,
                     vnode_augment)

__all__ = ["VfpiError", "load", "vfpi_create", "vfpi_destroy", "vfpi_error_string", "vfpi_step",
           "vfpi_step_backward", "vfpi_step_batched", "vfpi_tape_bytes", "Bsr", "Contacts", "Solver",
           "bsr_from_arrays", "contacts_from_arrays", "make_opts", "new_stats", "read_stats", "vnode_augment",
           "vfpi_vnode_pattern", "vfpi_vnode_values"]
