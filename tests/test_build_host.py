"""Host logic of the build: the spill check on kernels whose stage waits
count the loads a wave has in flight."""
from paper_2203_09353_amd import build

REMARKS = """\
bgemm_kernels.hip:722:1: remark: Function Name: _ZN2bg9k_uniformINS_3CfgILi128EEEvv [-Rpass-analysis=kernel-resource-usage]
bgemm_kernels.hip:722:1: remark:     VGPRs: 115 [-Rpass-analysis=kernel-resource-usage]
bgemm_kernels.hip:722:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
bgemm_kernels.hip:1109:1: remark: Function Name: _ZN2bg9k_vb_execINS_3CfgILi128EEEvv [-Rpass-analysis=kernel-resource-usage]
bgemm_kernels.hip:1109:1: remark:     VGPRs: 128 [-Rpass-analysis=kernel-resource-usage]
bgemm_kernels.hip:1109:1: remark:     ScratchSize [bytes/lane]: 64 [-Rpass-analysis=kernel-resource-usage]
bgemm_kernels.hip:858:1: remark: Function Name: _ZN2bg7k_scaleEdPKPdl [-Rpass-analysis=kernel-resource-usage]
bgemm_kernels.hip:858:1: remark:     ScratchSize [bytes/lane]: 16 [-Rpass-analysis=kernel-resource-usage]
"""


def test_spilling_counted_wait_kernel_is_reported():
    assert build.kernels_with_scratch(REMARKS) == ["_ZN2bg9k_vb_execINS_3CfgILi128EEEvv"]


def test_other_kernels_and_clean_builds_pass():
    clean = REMARKS.replace("ScratchSize [bytes/lane]: 64", "ScratchSize [bytes/lane]: 0")
    assert build.kernels_with_scratch(clean) == []
    assert build.kernels_with_scratch("") == []


def test_build_asks_the_compiler_for_resource_remarks():
    assert "-Rpass-analysis=kernel-resource-usage" in build.RESOURCE_REMARKS
    assert set(build.COUNTED_WAIT_KERNELS) == {"k_uniform", "k_vb_exec"}


def test_tuner_prefers_the_earlier_shape_on_a_tie():
    from paper_2203_09353_amd import tune
    order = ["a", "b", "c"]
    assert tune.pick({"a": 10.02, "b": 10.0, "c": 11.0}, order) == "a"     # within TIE
    assert tune.pick({"a": 10.5, "b": 10.0, "c": 11.0}, order) == "b"      # a clearly slower
    assert tune.pick({"b": 10.0, "c": 9.0}, order) == "c"                  # a not built
    assert tune.pick({"c": 9.0}, order) == "c"
