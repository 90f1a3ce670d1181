"""Host-side checks of the build script (no GPU): the resource-report parser that fails the
build when a kernel uses scratch memory."""
from paper_2512_12797_amd import build

REPORT = """\
x.hip:10:1: remark: Function Name: _Z3fooPf [-Rpass-analysis=kernel-resource-usage]
x.hip:10:1: remark:     VGPRs: 80 [-Rpass-analysis=kernel-resource-usage]
x.hip:10:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
x.hip:20:1: remark: Function Name: _Z3barPf [-Rpass-analysis=kernel-resource-usage]
x.hip:20:1: remark:     ScratchSize [bytes/lane]: 96 [-Rpass-analysis=kernel-resource-usage]
"""


def test_scratch_users_names_only_kernels_with_scratch():
    assert build.scratch_users(REPORT) == [("_Z3barPf", 96)]
    assert build.scratch_users(REPORT.replace("96", "0")) == []
