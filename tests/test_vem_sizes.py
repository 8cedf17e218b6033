"""The element's sizes from the library (a host query, no GPU) against the
generator's degree-of-freedom layout (Sec. 3, D1-D5), k = 2, 3, 4: the
numbering vb_vem_element_matrices writes its matrices in."""
import os

import pytest

from inputs.vem import DofLayout


@pytest.mark.parametrize("k", [2, 3, 4])
def test_vem_dofs_match_the_layout(k):
    from paper_2304_09770_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    n, p = binding.vb_vem_dofs(k)
    L = DofLayout(k)
    assert (n, p) == (L.N, L.nP)


def test_vem_dofs_rejects_other_degrees():
    from paper_2304_09770_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    with pytest.raises(binding.VBError):
        binding.vb_vem_dofs(5)
