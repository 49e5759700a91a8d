"""The allocation-free entry point dfdg_diagnostics_noalloc against dfdg_diagnostics.

Both run the same kernels; only the scratch differs (the library's static device array
instead of the context's workspace), so the four numbers must agree bit for bit.  Two
calls in a row on different contexts share the array, the second on a smaller mesh.
"""
import pytest

from inputs import double_shear_layer, eval_broken_poly, random_broken_poly

pytestmark = pytest.mark.gpu

from gpu_util import make_pair, project_field, values_to_lib  # noqa: E402


def test_noalloc_diagnostics_equal_the_workspace_ones():
    results = []
    for n, k, kind in ((48, 2, "dsl"), (7, 1, "broken")):
        print("noalloc diagnostics: mesh", n, "k", k, kind, flush=True)
        _, s, xyz, _ = make_pair(n, k, oracle=False, precond="amg", cg_rtol=1e-12)
        if kind == "dsl":
            U, _ = project_field(s, xyz, double_shear_layer)
        else:
            coef = random_broken_poly(s.T, k, seed=3)
            U = values_to_lib(s, lambda pts: eval_broken_poly(coef, pts))
        ref = s.diagnostics(U)
        got = s.diagnostics_noalloc(U)
        print("  workspace", ref, "\n  static   ", got, flush=True)
        assert got == ref
        assert ref["energy"] > 0 and ref["enstrophy"] > 0
        results.append(got)
        del s
    assert results[0] != results[1]
