"""Host-side helpers of the profile summaries (no GPU)."""
from paper_2210_12252_amd.profiling import short_name


def test_short_name_keeps_template_and_namespace():
    assert short_name("void helic::k_radial_inverse<double, 12>(double const*, long, double*)") == \
        "helic::k_radial_inverse<double, 12>"


def test_short_name_drops_anonymous_namespace():
    # kernels in an anonymous namespace must not collapse into one "helic::" row
    n1 = short_name("helic::(anonymous namespace)::k_cheb_step(double const*, double const*, double*, long)")
    n2 = short_name("helic::(anonymous namespace)::k_residual(double const*, double const*, double const*)")
    assert n1 == "helic::k_cheb_step" and n2 == "helic::k_residual"
