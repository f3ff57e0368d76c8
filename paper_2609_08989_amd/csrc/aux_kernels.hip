// aux_kernels.hip -- small device kernels: buffer fills (used instead of
// hipMemsetAsync so that the same code is safe inside captured graphs) and the
// analytic Kerr table builder for the tabulated-metric path.
#include <hip/hip_runtime.h>

#include <cmath>

namespace tartarus {

__global__ void fill_u32_kernel(unsigned int* p, unsigned int v, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void fill_u64_kernel(unsigned long long* p, unsigned long long v, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// Kerr components in the tabulated (smooth) form and their exact derivatives
// d/dr, d/dtheta, d2/dr dtheta, from the closed forms
//   u = 2r / Sigma,  g_tt = u - 1,  g_tphi / s^2 = -a u,  g_rr = Sigma / Delta,
//   g_thth = Sigma,  g_phph / s^2 = r^2 + a^2 + a^2 s^2 u,
// with Sigma_r = 2r, Sigma_th = -2 a^2 s c, Delta_r = 2r - 2.
__global__ void build_kerr_table_kernel(double a, int nr, int nth, double u0, double du, double dth, double* tab)
{
    const long long n = (long long)nr * nth;
    const long long plane = n * 4;
    for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int k = (int)(idx / nth), l = (int)(idx % nth);
        const double r = exp(u0 + (double)k * du);
        const double th = (double)l * dth;
        double s, c;
        sincos(th, &s, &c);
        const double a2 = a * a, r2 = r * r, s2 = s * s;
        const double sig = r2 + a2 * c * c;
        const double del = r2 - 2.0 * r + a2;
        const double isg = 1.0 / sig;
        const double sig_t = -2.0 * a2 * s * c;
        const double u = 2.0 * r * isg;
        const double u_r = 2.0 * isg - 4.0 * r2 * isg * isg;
        const double u_t = -2.0 * r * sig_t * isg * isg;
        const double u_rt = sig_t * (-2.0 * isg * isg + 8.0 * r2 * isg * isg * isg);
        const double idel = 1.0 / del;
        double v[5][4];
        v[0][0] = u - 1.0;  v[0][1] = u_r;       v[0][2] = u_t;       v[0][3] = u_rt;
        v[1][0] = -a * u;   v[1][1] = -a * u_r;  v[1][2] = -a * u_t;  v[1][3] = -a * u_rt;
        v[2][0] = sig * idel;
        v[2][1] = (2.0 * r * del - sig * (2.0 * r - 2.0)) * idel * idel;
        v[2][2] = sig_t * idel;
        v[2][3] = -sig_t * (2.0 * r - 2.0) * idel * idel;
        v[3][0] = sig;      v[3][1] = 2.0 * r;   v[3][2] = sig_t;     v[3][3] = 0.0;
        v[4][0] = r2 + a2 + a2 * s2 * u;
        v[4][1] = 2.0 * r + a2 * s2 * u_r;
        v[4][2] = a2 * (2.0 * s * c * u + s2 * u_t);
        v[4][3] = a2 * (2.0 * s * c * u_r + s2 * u_rt);
        for (int comp = 0; comp < 5; ++comp) {
            double* e = tab + comp * plane + idx * 4;
            e[0] = v[comp][0];
            e[1] = v[comp][1];
            e[2] = v[comp][2];
            e[3] = v[comp][3];
        }
    }
}

}  // namespace tartarus

using namespace tartarus;

static int blocks_for(long long n, int threads)
{
    long long b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > 65536) b = 65536;
    return (int)b;
}

extern "C" hipError_t tartarus_launch_fill_u32(unsigned int* p, unsigned int v, long long n, hipStream_t stream)
{
    hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, stream, p, v, n);
    return hipGetLastError();
}

extern "C" hipError_t tartarus_launch_fill_u64(unsigned long long* p, unsigned long long v, long long n,
                                               hipStream_t stream)
{
    hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, stream, p, v, n);
    return hipGetLastError();
}

extern "C" hipError_t tartarus_launch_build_table(double a, int nr, int nth, double r_min, double r_max, double* table,
                                                  hipStream_t stream)
{
    const double u0 = log(r_min);
    const double du = (log(r_max) - log(r_min)) / (double)(nr - 1);
    const double dth = M_PI / (double)(nth - 1);
    hipLaunchKernelGGL(build_kerr_table_kernel, dim3(blocks_for((long long)nr * nth, 256)), dim3(256), 0, stream, a, nr,
                       nth, u0, du, dth, table);
    return hipGetLastError();
}
