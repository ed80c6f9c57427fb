"""Each pin of tests/test_oracle_pins.py must catch a plausible mistake.

For every entry below a copy of the oracle's C sources is built with one
planted mistake (a dropped factor, a swapped or mis-signed coefficient, a
changed constant), and the named pin is run against that copy through
oracle.using_library: it must fail.  The copies live in a temporary
directory; the oracle itself is not touched."""
import concurrent.futures as cf
import os
import shutil

import pytest

import oracle
from oracle import build as oracle_build
import test_oracle_pins as pins
import test_oracle_shade as shade_pins

ORACLE_DIR = os.path.dirname(oracle.__file__)

# name: (file, [(text, replacement), ...], pin to run against the copy)
MUTATIONS = {
    "smith_lambda_without_half": (
        "shade.c", [("return 0.5 * (-1.0 + sqrt(1.0 + a2 * tan2));", "return (-1.0 + sqrt(1.0 + a2 * tan2));")],
        lambda: pins.test_ggx_visible_normal_identity(0.5, 1.2)),
    "schlick_f0_0p4": (
        "shade.c", [("out[4] = 0.04 + 0.96 * pow(", "out[4] = 0.4 + 0.6 * pow(")],
        pins.test_schlick_fresnel_limits),
    "shadowing_uncorrelated": (
        "shade.c", [("out[3] = 1.0 / (1.0 + out[1] + out[2]);", "out[3] = 1.0 / ((1.0 + out[1]) * (1.0 + out[2]));")],
        lambda: pins.test_ggx_shadowing_is_height_correlated(0.6)),
    "lobe_over_2_not_4": (
        "shade.c", [("/ (4.0 * no * ni);", "/ (2.0 * no * ni);")],
        lambda: pins.test_shading_weak_white_furnace(0.15, 0.6)),
    "ewa_A_and_C_swapped": (
        "oracle.c", [("float A = (d0y * d0y + d1y * d1y) + 1.0f;", "float A = (d0x * d0x + d1x * d1x) + 1.0f;"),
                     ("float Cc = (d0x * d0x + d1x * d1x) + 1.0f;", "float Cc = (d0y * d0y + d1y * d1y) + 1.0f;")],
        lambda: pins.test_ewa_ellipse_second_moments(6.0, 1.5, 0.0)),
    "ewa_B_sign": (
        "oracle.c", [("float B = -2.0f * (d0x * d0y + d1x * d1y);", "float B = 2.0f * (d0x * d0y + d1x * d1y);")],
        lambda: pins.test_ewa_ellipse_second_moments(8.0, 2.0, 0.5)),
    "ewa_without_texel_widening": (
        "oracle.c", [("float A = (d0y * d0y + d1y * d1y) + 1.0f;", "float A = (d0y * d0y + d1y * d1y) + 0.0f;"),
                     ("float Cc = (d0x * d0x + d1x * d1x) + 1.0f;", "float Cc = (d0x * d0x + d1x * d1x) + 0.0f;")],
        lambda: pins.test_ewa_ellipse_second_moments(0.5, 0.25, 0.0)),
    "pcg_increment": (
        "oracle.c", [("uint32_t state = x * 747796405u + 2891336453u;", "uint32_t state = x * 747796405u + 2891336451u;")],
        pins.test_pcg_known_answers),
    "chain_axis0_unhashed": (
        "oracle.c", [("uint32_t h = orc_pcg(b + axis);", "uint32_t h = axis ? orc_pcg(b + axis) : b;")],
        pins.test_uniform_known_answers),
    "breakpoint_c2_without_c1": (
        "oracle.c", [("c[1] = c[0] + (4.0f + (3.0f * (t * t)) * (t - 2.0f)) * K6;",
                      "c[1] = (4.0f + (3.0f * (t * t)) * (t - 2.0f)) * K6;")],
        pins.test_cubic_breakpoints_known_answers),
    "material_normal_components_swapped": (
        "shade.c", [("    out[4] = orc_h2d(hx);\n    out[5] = orc_h2d(hy);", "    out[4] = orc_h2d(hy);\n    out[5] = orc_h2d(hx);")],
        lambda: shade_pins.test_material_source_stochastic_reads_the_decoded_texel(oracle.CUBIC)),
    "material_unorm_over_256": (
        "shade.c", [("out[0] = texel[0] / 255.0;", "out[0] = texel[0] / 256.0;")],
        lambda: shade_pins.test_material_source_stochastic_reads_the_decoded_texel(oracle.LINEAR)),
    "material_texels_transposed": (
        "oracle.c", [("orc_material_decode((const uint8_t*)s->tex + 8 * ((int64_t)y * s->W + x), m);",
                      "orc_material_decode((const uint8_t*)s->tex + 8 * ((int64_t)x * s->H + y), m);")],
        lambda: shade_pins.test_material_source_deterministic_matches_decoded_texture(oracle.CUBIC)),
    "cubic_taps_not_centred": (
        "oracle.c", [("    int j = (u >= c[0]) + (u >= c[1]) + (u >= c[2]);\n    return j - 1;",
                      "    int j = (u >= c[0]) + (u >= c[1]) + (u >= c[2]);\n    return j;")],
        pins.test_tap_known_answers),
}


def _build_mutant(root, name):
    fname, edits, _ = MUTATIONS[name]
    d = os.path.join(root, name)
    os.makedirs(d)
    for f in oracle_build.SOURCES:
        src = os.path.join(ORACLE_DIR, f)
        if os.path.exists(src):
            shutil.copy(src, d)
    path = os.path.join(d, fname)
    text = open(path).read()
    for old, new in edits:
        assert text.count(old) == 1, f"{name}: '{old}' is not unique in {fname}"
        text = text.replace(old, new)
    open(path, "w").write(text)
    return oracle_build.build(src_dir=d, target=os.path.join(d, "liboracle.so"))


@pytest.fixture(scope="module")
def mutants(tmp_path_factory):
    root = str(tmp_path_factory.mktemp("oracle_mutants"))
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        paths = dict(zip(MUTATIONS, ex.map(lambda n: _build_mutant(root, n), MUTATIONS)))
    return paths


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pin_catches_planted_mistake(name, mutants):
    pin = MUTATIONS[name][2]
    with oracle.using_library(mutants[name]):
        with pytest.raises(AssertionError):
            pin()
    pin()   # and passes again on the oracle itself
