"""Error paths of the C ABI that fail before any device work: NULL handles
and outputs, a device that does not exist.  They run on a machine without
a GPU (no kernel is launched)."""

import ctypes as C

from paper_2209_13168_amd import ecmd


def test_null_handles_and_outputs_are_rejected():
    L = ecmd.lib()
    sen = ecmd.sensor(64, 48, (32, 24))
    sp = ecmd._search(0.0, 1.0, 1e-3)
    res = (ecmd.ResultS * 1)()
    assert L.ecmd_ctx_create(None, 0, None) == ecmd.EINVAL
    assert L.ecmd_estimate_divergence_batched(None, C.byref(sen), None, None, None, None, None, 1, C.byref(sp), 0,
                                              None, res) == ecmd.EINVAL
    assert L.ecmd_plan_create(None, C.byref(sen), C.byref(sp), None, None) == ecmd.EINVAL
    assert L.ecmd_plan_launch(None, None, None, None, None, None, None, 1, None, None) == ecmd.EINVAL
    assert L.ecmd_cnn_create(None, C.c_uint64(0), None) == ecmd.EINVAL
    assert L.ecmd_cnn_save(None, b"x") == ecmd.EINVAL
    assert L.ecmd_cnn_load(None, b"x") == ecmd.EINVAL
    assert L.ecmd_ctx_set_profiling(None, 1) == ecmd.EINVAL
    assert L.ecmd_ctx_get_profile(None, None, 0) == ecmd.EINVAL
    assert L.ecmd_last_error(None) == b"NULL context"
    # destroying nothing is a no-op
    L.ecmd_ctx_destroy(None)
    L.ecmd_plan_destroy(None)
    L.ecmd_cnn_destroy(None)


def test_missing_device_is_a_device_error():
    h = C.c_void_p()
    rc = ecmd.lib().ecmd_ctx_create(C.byref(h), 4096, None)
    assert rc == ecmd.EDEVICE and not h.value
