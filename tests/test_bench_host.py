"""Host-side helpers of bench.py (no GPU): the algorithmic byte counts of
the passes against the closed forms of the schedule, the tile decoding of
kernel-trace records (including the one-dimensional column grids with edge
workgroups), and the schedule descriptions."""
import bench


def _n(nx, ny, nz):
    return nx * ny * nz


def test_demag_bytes_match_the_closed_form():
    # a 3-D demag moves ~336 N bytes: with N' = 3 nz ny (nx + 1) complex
    # elements of X1 and 2N' of X2, x forward 12N + 8N', y forward 8N' + 16N',
    # z product 2 x 16N' + the K~ octant, y inverse 16N' + 8N', x inverse
    # 8N' + 12N
    nx = ny = nz = 64
    N = _n(nx, ny, nz)
    nc = 3 * nz * ny * (nx + 1)
    nK = 6 * (nz + 1) * (ny + 1) * (nx + 1)
    b = bench.pass_bytes(nx, ny, nz)
    demag = b["xfwd"] + b["yfwd"] + b["zconv"] + b["yinv"] + b["xinv"]
    assert demag == 24 * N + 96 * nc + 4 * nK
    assert 330 < demag / N < 345


def test_fused_step_saves_the_field_round_trip():
    nx, ny, nz = 128, 128, 128
    N = _n(nx, ny, nz)
    nc = 3 * nz * ny * (nx + 1)
    unfused = bench.step_bytes(nx, ny, nz, fused=False)
    fused = bench.step_bytes(nx, ny, nz, fused=True)
    # per stage the fused pass drops the field's write and read (24N), the
    # stage kernel's re-read of the new state by the next x forward (12N),
    # except after stage 4, and three of the four x forwards
    b = bench.pass_bytes(nx, ny, nz)
    assert unfused - fused == 3 * b["xfwd"] + 4 * b["xinv"] + 4 * b["stage"] - 4 * b["xstage"]
    assert 1590 < unfused / N < 1615
    assert fused < unfused
    # the per-stage table of the fused pass averages to its per-launch figure
    per_stage = [a * N + c * nc for a, c in bench.XSTAGE_BYTES.values()]
    assert sum(per_stage) / 4.0 == b["xstage"]


def test_trace_records_decode_to_pass_and_tile():
    shape = (128, 128, 128)
    nx, ny, nz = shape
    pairs = (3 * nz * ny + 1) // 2
    # x forward, 16 row pairs per workgroup, variant 2
    k = "void mmk::k_xfwd<256, 2>(float const*, HIP_vector_type<float, 2u>*, int, int, int, HIP_vector_type<float, 2u> const*)"
    assert bench.pass_tile_of(k, -(-pairs // 16), 0, shape) == ("xfwd", 16 + 512, 0)
    # y forward with P = 8: 16 tiles of the 128 columns below Lx/2 per plane
    # plus edge workgroups for the last column, 8 planes each
    k = "void mmk::k_yfwd<256, 0>(HIP_vector_type<float, 2u> const*, HIP_vector_type<float, 2u>*, int, int, int)"
    nrows = 3 * nz
    blocks = (nx // 8) * nrows + -(-nrows // 8)
    assert bench.pass_tile_of(k, blocks, 0, shape) == ("yfwd", 8, 0)
    # z product, P = 16 in radix order 1 (variant 3), rows = Ly = 2 ny
    k = "void mmk::k_conv_reg3<256, true, 1>(HIP_vector_type<float, 2u>*, float const*, int, int, int, int)"
    blocks = (nx // 16) * 2 * ny + -(-2 * ny // 16)
    assert bench.pass_tile_of(k, blocks, 0, shape) == ("zconv", 16 + 3 * 256, 0)
    # the fused stage pass: P = 2 row pairs (2P rows per workgroup), W = 1, RK4 stage 3
    k = "void mmk::k_xstage<256, 3, true, 1>(HIP_vector_type<float, 2u>*, float const*, float const*, float*, float*)"
    assert bench.pass_tile_of(k, nz * ny // 4, 0, shape) == ("xstage", 2, 3)
    # another transform length is not this grid's pass
    k = "void mmk::k_yfwd<128, 0>(HIP_vector_type<float, 2u> const*, HIP_vector_type<float, 2u>*, int, int, int)"
    assert bench.pass_tile_of(k, 100, 0, shape) is None


def test_schedule_descriptions():
    d = bench.describe_tiles({"xfwd": 528, "zconv": 16, "yconv": 0, "stage": 4, "reduce": 0, "xstage": 2})
    assert "radix order 1" in d["xfwd"] and d["xfwd"].startswith("16 row pairs")
    assert d["zconv"] == "16 columns per workgroup, three components in registers, default radix order"
    assert "yconv" not in d and "reduce" not in d
    assert d["stage"] == "4 cells per thread"
    assert d["xstage"].startswith("fused") and "2 row pairs" in d["xstage"]
    assert bench.describe_tiles({"xstage": 0}) == {}


def test_mangled_kernel_names_are_shortened():
    # the trace can leave a kernel with a bf16 parameter mangled
    assert bench._demangle_mmk("_ZN3mmk9k_conv_inILi3EEEvPKDF16bS2_PKfPDF16bS5_S5_NS_7PadGeomEiii") == "mmk::k_conv_in<3>"
    assert bench._demangle_mmk(
        "_ZN3mmk6k_convILi0ELb1ELb0EEEvPKDF16bS2_PKfPfPDF16bS6_S5_fS4_iiiiiS6_NS_7PadGeomE") == "mmk::k_conv<0, true, false>"
    assert bench._demangle_mmk("_ZN3mmk5k_mseEPKfS1_fPDF16bS2_NS_7PadGeomEPd") == "mmk::k_mse"
    assert bench._demangle_mmk("void mmk::k_adam(float*)") == "void mmk::k_adam(float*)"


def test_surrogate_counter_summary_from_synthetic_databases(tmp_path):
    # two counter databases in the layout rocprofv3 writes (one row per
    # dispatch, kernel and counter, per shader engine here: summed), one
    # convolution with two dispatches and one other kernel that is left out
    import sqlite3
    vals = {"SQ_WAVES": 4096, "SQ_INSTS_VALU": 4096 * 680, "SQ_INSTS_MFMA": 4096 * 180, "SQ_INSTS_LDS": 4096 * 61,
            "SQ_INSTS_VMEM_RD": 4096 * 45, "SQ_WAVE_CYCLES": 1000000, "SQ_BUSY_CYCLES": 50000,
            "SQ_VALU_MFMA_BUSY_CYCLES": 1024 * 2400 * 4.8, "SQ_ACTIVE_INST_VALU": 1, "SQ_ACTIVE_INST_LDS": 400,
            "SQ_LDS_BANK_CONFLICT": 1000, "SQ_WAIT_INST_ANY": 300000, "SQ_WAIT_ANY": 500000,
            "SQ_ACTIVE_INST_ANY": 200000}
    conv = "_ZN3mmk6k_convILi3ELb1ELb1EEEvPKDF16bS2_PKfPfPDF16bS6_S5_fS4_iiiiiS6_NS_7PadGeomE"
    for kind, names in bench.SUR_SQ_SETS.items():
        d = tmp_path / kind / "host"
        d.mkdir(parents=True)
        con = sqlite3.connect(str(d / "x_results.db"))
        con.execute("create table counters_collection (dispatch_id int, kernel_name text, counter_name text, "
                    "value real)")
        for disp in (1, 2):
            for c in names:
                for se in range(2):  # two halves that the summary adds up
                    con.execute("insert into counters_collection values (?, ?, ?, ?)", (disp, conv, c, vals[c] / 2))
        con.execute("insert into counters_collection values (3, 'void mmk::k_adam(float*)', 'SQ_WAVES', 4)")
        con.commit()
        con.close()
    text = bench.summarize_surrogate_counters(str(tmp_path))
    rows = [ln for ln in text.splitlines() if ln.startswith("mmk::")]
    assert len(rows) == 1 and rows[0].startswith("mmk::k_conv<3, true, true>")
    f = rows[0][30:].split()
    assert f[:5] == ["4096", "680", "180", "61", "45.0"]
    assert f[5] == "4.80" and f[6] == "2.500"
    assert f[7:] == ["0.300", "0.500", "0.200"]
    assert "--summarize-surrogate-counters" in text
