"""CPU check that every family of the mixed launch has its kernel: the
library's own consistency check, run without a GPU (it resolves the kernel
of each family and reports the first family without one)."""
from paper_2310_16214_amd import ppx


def test_every_family_has_a_kernel():
    assert ppx.lib().ppx_mixed_families_complete() == 0, ppx.last_error()
