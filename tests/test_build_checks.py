"""The build's check that no kernel uses scratch (per-lane private memory),
read from the compiler's resource-usage remarks."""
from paper_1706_06940_amd.build import scratch_kernels

REMARKS = """\
x.hip:5:1: remark: Function Name: k_one [-Rpass-analysis=kernel-resource-usage]
x.hip:5:1: remark:     VGPRs: 14 [-Rpass-analysis=kernel-resource-usage]
x.hip:5:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
x.hip:9:1: remark: Function Name: k_two [-Rpass-analysis=kernel-resource-usage]
x.hip:9:1: remark:     ScratchSize [bytes/lane]: 20 [-Rpass-analysis=kernel-resource-usage]
x.hip:12:1: remark: Function Name: k_three [-Rpass-analysis=kernel-resource-usage]
x.hip:12:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
"""


def test_scratch_kernels_names_only_the_spilling_ones():
    assert scratch_kernels(REMARKS) == [("k_two", 20)]


def test_no_remarks_no_findings():
    assert scratch_kernels("") == []
    assert scratch_kernels(REMARKS.replace(": 20 ", ": 0 ")) == []
