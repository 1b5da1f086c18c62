"""Launch geometry on the host (no GPU): every launch the library issues, enumerated workgroup by
workgroup for the colour passes, up to and beyond the Table 7 sizes.

For every (dim, degree) and every level whose node count N = (k 2^L + 1)^d stays below 2^31 (3D Q1 at
1025^3, 3D Q3 at 1537^3 and 3D Q7 at 897^3 included), vps_launch_geometry_check must find every
colour-pass workgroup of every colour and launch shape on patches of its colour inside the grid,
each patch covered once, closure offsets within 32 bits, and every operator and transfer launch
within its launcher's limits.  Past the 32-bit limits the check (and the launchers) must refuse."""
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2405_19004_amd", "libvps.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libvps.so not built")


def _levels(d, k, limit=2 ** 31):
    L = 1
    while (k * 2 ** L + 1) ** d < limit:
        yield L
        L += 1


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("k", range(1, 8))
def test_every_launch_fits_up_to_two_billion_nodes(d, k):
    import paper_2405_19004_amd as v
    top = max(_levels(d, k))
    blocks = v.vps_launch_geometry_check(d, k, top)  # checks levels 1..top
    assert blocks > 0


@pytest.mark.parametrize("d,k,L", [(3, 1, 9), (3, 3, 8), (3, 7, 7), (3, 4, 6), (2, 7, 9), (3, 3, 5)])
def test_workload_and_table7_hierarchies(d, k, L):
    import paper_2405_19004_amd as v
    assert v.vps_launch_geometry_check(d, k, L) > 0


@pytest.mark.parametrize("d,k,L", [(3, 7, 10), (3, 4, 11), (2, 7, 17)])
def test_beyond_the_offset_limits_is_refused(d, k, L):
    import paper_2405_19004_amd as v
    with pytest.raises(v.VpsError) as e:
        v.vps_launch_geometry_check(d, k, L)
    assert e.value.status == v.VPS_EINVAL and "level" in str(e.value)
