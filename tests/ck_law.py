"""The exact survival of static targets among independent mobile B's (Collins-Kimball), the
expected value of the Collins-Kimball pins."""
import math

from scipy import integrate, special


def ck_survival(t, rho, D, sigma, kappa):
    """exp(-rho int_0^t k(s) ds) with the time-dependent Collins-Kimball rate
    k(s) = k_CK [1 + (kappa/k_D) e^{a^2 D s} erfc(a sqrt(D s))], k_D = 4 pi sigma D,
    k_CK = kappa k_D / (kappa + k_D), a = (1 + kappa/k_D) / sigma: a static target's survival
    among independent B's of density rho diffusing with D (radiation surface at sigma)."""
    kD = 4.0 * math.pi * sigma * D
    kck = kappa * kD / (kappa + kD)
    a = (1.0 + kappa / kD) / sigma

    def k(s):
        return kck * (1.0 + (kappa / kD) * special.erfcx(a * math.sqrt(D * s)))

    return math.exp(-rho * integrate.quad(k, 0.0, t, limit=400, epsabs=0.0, epsrel=1e-12)[0])
