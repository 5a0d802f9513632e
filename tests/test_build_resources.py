"""The build's kernel resource check: parsing of the compiler's per-kernel
resource remarks, and the rules (no scratch, two wavefronts per SIMD for the
body-schedule rollout kernel and the persistent kernels)."""
import pytest

from paper_2511_19204_amd import build

REMARKS = """
k.hip:10:1: remark: Function Name: _ZN4mppi14rollout_kernelILi16EEEvPKi [-Rpass-analysis=kernel-resource-usage]
k.hip:10:1: remark:     TotalSGPRs: 106 [-Rpass-analysis=kernel-resource-usage]
k.hip:10:1: remark:     VGPRs: 253 [-Rpass-analysis=kernel-resource-usage]
k.hip:10:1: remark:     AGPRs: 0 [-Rpass-analysis=kernel-resource-usage]
k.hip:10:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
k.hip:10:1: remark:     Occupancy [waves/SIMD]: 2 [-Rpass-analysis=kernel-resource-usage]
k.hip:20:1: remark: Function Name: _ZN4mppi25rollout_persistent_kernelILi16EEEvPKi [-Rpass-analysis=kernel-resource-usage]
k.hip:20:1: remark:     VGPRs: 256 [-Rpass-analysis=kernel-resource-usage]
k.hip:20:1: remark:     AGPRs: 0 [-Rpass-analysis=kernel-resource-usage]
k.hip:20:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
k.hip:20:1: remark:     Occupancy [waves/SIMD]: 2 [-Rpass-analysis=kernel-resource-usage]
k.hip:30:1: remark: Function Name: _ZN4mppi11team_kernelILi16EEEvPKi [-Rpass-analysis=kernel-resource-usage]
k.hip:30:1: remark:     VGPRs: 256 [-Rpass-analysis=kernel-resource-usage]
k.hip:30:1: remark:     AGPRs: 12 [-Rpass-analysis=kernel-resource-usage]
k.hip:30:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
k.hip:30:1: remark:     Occupancy [waves/SIMD]: 1 [-Rpass-analysis=kernel-resource-usage]
"""


def test_remarks_are_parsed_per_kernel():
    u = build.resource_usage(REMARKS)
    assert u["_ZN4mppi14rollout_kernelILi16EEEvPKi"] == {"VGPRs": 253, "AGPRs": 0, "ScratchSize": 0, "Occupancy": 2}
    assert u["_ZN4mppi25rollout_persistent_kernelILi16EEEvPKi"]["Occupancy"] == 2
    assert u["_ZN4mppi11team_kernelILi16EEEvPKi"]["AGPRs"] == 12


def test_rules():
    build.check_resources(build.resource_usage(REMARKS))  # other kernels may run one wavefront per SIMD
    low = REMARKS.replace("Occupancy [waves/SIMD]: 2", "Occupancy [waves/SIMD]: 1", 1)
    with pytest.raises(RuntimeError, match="rollout_kernel.*occupancy"):
        build.check_resources(build.resource_usage(low))
    low_p = REMARKS.replace("Occupancy [waves/SIMD]: 2 [-Rpass-analysis=kernel-resource-usage]\nk.hip:30",
                            "Occupancy [waves/SIMD]: 1 [-Rpass-analysis=kernel-resource-usage]\nk.hip:30", 1)
    assert low_p != REMARKS
    with pytest.raises(RuntimeError, match="persistent_kernel.*occupancy"):
        build.check_resources(build.resource_usage(low_p))
    spill = REMARKS.replace("ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]\nk.hip:20",
                            "ScratchSize [bytes/lane]: 48 [-Rpass-analysis=kernel-resource-usage]\nk.hip:20", 1)
    with pytest.raises(RuntimeError, match="scratch"):
        build.check_resources(build.resource_usage(spill))
    with pytest.raises(RuntimeError, match="no kernel"):
        build.check_resources({})
