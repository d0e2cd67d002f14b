"""The pins are strong enough: plausible mistakes planted in the oracle (on
the CPU, by monkeypatching one helper at a time) each make at least one pin
fail."""
import numpy as np
import pytest

import oracle.core as core
import tests.test_oracle_adjoint as tadj
import tests.test_oracle_vfpi as tv

_orig_project = core.project_strict
_orig_jac = core.contact_jacobian
_orig_w = core.frobenius_w


def _proj_radius_mu(lam_star, mu):            # disk radius mu instead of mu * lambda_n
    ls = np.asarray(lam_star, dtype=np.float64).copy()
    lam, br = _orig_project(ls, mu / np.maximum(np.maximum(ls[:, 0], 0), 1e-300))
    return lam, br


def _proj_no_clamp(lam_star, mu):             # normal impulse not clamped at zero
    lam, br = _orig_project(lam_star, mu)
    neg = lam_star[:, 0] < 0
    lam[neg, 0] = lam_star[neg, 0]
    return lam, br


def _jac_transposed(p):                       # R^T instead of R in eq. jcnode
    q = core.__dict__["_Tmp"](p)
    return _orig_jac(q)


def _w_unsquared(p, diag, rn2):               # ||A_d*||_2 instead of its square
    return _orig_w(p, diag, np.sqrt(rn2))


def _w_no_groups(p, diag, rn2):               # per-DOF values even on contact nodes
    return diag / rn2


class _T:
    def __init__(self, p):
        self.__dict__.update(p.__dict__)
        self.R = p.R.transpose(0, 2, 1).copy()

    def __getattr__(self, k):
        raise AttributeError(k)

    @property
    def n(self):
        return 3 * self.n_nodes

    @property
    def n_contacts(self):
        return self.c_node.shape[0]


PINS = [
    lambda: tv.test_inclined_plane_threshold_analytic(0.0),
    lambda: tv.test_inclined_plane_threshold_analytic(0.3),
    lambda: tv.test_prop4_surrogate_scc_exact_every_sweep(0),
    lambda: [tv.test_frictionless_matches_lcp_enumeration(s) for s in range(2)],
    lambda: tv.test_cloth10_matches_pgs(),
    lambda: tv.test_one_to_three_contacts_match_mode_enumeration(2, 2),
    lambda: tadj.test_sliding_particle_closed_form(),
    lambda: tv.test_tangent_basis_invariance(),
]


@pytest.mark.parametrize("name,target,mutant", [
    ("radius", "project_strict", _proj_radius_mu),
    ("noclamp", "project_strict", _proj_no_clamp),
    ("transposedR", "contact_jacobian", _jac_transposed),
    ("unsquared", "frobenius_w", _w_unsquared),
    ("nogroups", "frobenius_w", _w_no_groups),
])
def test_planted_mistake_is_caught(monkeypatch, name, target, mutant):
    monkeypatch.setattr(core, "_Tmp", _T, raising=False)
    monkeypatch.setattr(core, target, mutant)
    failed = 0
    for pin in PINS:
        try:
            pin()
        except (AssertionError, ValueError, np.linalg.LinAlgError):
            failed += 1
    assert failed >= 1, f"mutant {name} survived every pin"
